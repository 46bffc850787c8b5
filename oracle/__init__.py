"""FP64 CPU oracle of the k-space pseudospectral time-reversal gradient.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import, call or execute anything in this package.  The product
(``paper_2102_00755_amd``) never imports it, and this package never imports
the product: the two share no code except the seeded input generators in
``synth`` (which hold none of the method's arithmetic).

Method: Lucka, Perez-Liva, Treeby, Cox, "High Resolution 3D Ultrasonic
Breast Imaging by Time-Domain Full Waveform Inversion", arXiv 2102.00755,
Appendix B (k-space pseudospectral scheme, eq. DisPartDev / DisPartDevSt,
Algorithm 1) and Sec. 2.3 (eq. Gradc0), Sec. 3.1 (eq. TRBwdWave), Sec. 3.2 /
App. E (source encoding).

Every function here is pinned by a ``-m "not gpu"`` test against something
other than itself (brute-force DFT, the closed-form single-mode evolution,
the homogeneous Green's function, exact reversibility, linearity,
finite differences, the dot-product test, published SplitMix64 outputs).
``oracle.slbfgs`` holds the stochastic L-BFGS of App. D (Algorithm 2), pinned
by tests/test_oracle_slbfgs.py; ``oracle.multigrid`` the grid transfers of
App. C, pinned by tests/test_oracle_multigrid.py; ``oracle.lossy`` the
power-law absorption of Sec. 2.1 (lossy forward, TR with the absorption sign
switched, exact lossy gradient), pinned by tests/test_oracle_lossy.py.

Parity unpinned: the absolute PML profile and the source pulse shape are
definitions of this build (the paper gives neither); they are checked only
for their qualitative property (the PML absorbs) and matched oracle <-> GPU.
"""

from .kspace import (  # noqa: F401
    Scheme,
    State,
    rademacher,
    delays,
    delayed_signals,
    splitmix64,
    forward,
    tr_gradient,
    full_gradient,
    exact_adjoint_gradient,
    tangent_linear_traces,
    misfit_and_adjoint_source,
    brute_force_dft3,
)
