"""Host logic of bench.py: the algorithmic bytes per cell-step of the time
step, at the limiting cases of the compact split-density storage.

Without PML every x-line keeps only the undamped density sum and one
spectrum of d-_y v_y + d-_z v_z: 32 + 0 + 2 = 34 field accesses = 136 B.
With every line in a y or z PML slab (and every x pair in the x PML) the
storage is the full split: 32 + 2 + 6 = 40 = 160 B, the eight-pass step.
"""

import bench


def test_step_bytes_limits():
    assert bench.step_bytes_per_cell((8, 8, 16), (0, 0, 0)) == 4.0 * 34
    # P = n / 2 on y and z puts every line in a slab; P = nx / 2 every x pair in the x PML
    assert bench.step_bytes_per_cell((8, 8, 16), (8, 4, 4)) == 4.0 * 40


def test_step_bytes_full_workload():
    # 448 x 448 x 224, PML 20: f = 1 - 408 * 184 / (448 * 224) of the lines in a
    # slab, 20 x-PML pairs per line (P even: no pair straddles the edge)
    f = 1.0 - 408 * 184 / (448 * 224)
    rho = 6.0 * f + (2.0 + 4.0 * 20 / 448) * (1.0 - f)
    want = 4.0 * (32.0 + 2.0 * f + rho)
    got = bench.step_bytes_per_cell((224, 448, 448), (20, 20, 20))
    assert abs(got - want) < 1e-9 and abs(got - 142.58) < 0.01
