// Host side of the C-ABI (include/fwi.h): handle, operator tables, geometry
// tables, workspace and the time loops of Alg. 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fwi.h"
#include "dispatch.h"
#include "exact_kernels.h"
#include "optim_kernels.h"

using namespace fwi;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define FWI_HIP(call)                                                                \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(FWI_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

constexpr double kPi = 3.14159265358979323846264338327950288;

// signed FFT frequency index (numpy fftfreq convention)
inline int signed_freq(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// PML multiplier Lambda = exp(-alpha_pml (c_ref/dx) (d/P)^4 dt / 2) (App. B),
// d = distance in cells into a PML of P cells; staggered points at i + 1/2.
std::vector<double> pml_profile(int n, int P, double dx, double dt, double c_ref, double alpha, bool stag) {
  std::vector<double> out(n, 1.0);
  if (P == 0) return out;
  for (int i = 0; i < n; ++i) {
    const double s = i + (stag ? 0.5 : 0.0);
    const double d = std::max(0.0, std::max(P - s, s - (n - 1 - P)));
    const double a = alpha * (c_ref / dx) * std::pow(d / P, 4.0);
    out[i] = std::exp(-a * dt / 2.0);
  }
  return out;
}

struct Geometry {
  int nlines = 0;
  std::vector<int32_t> src_off, rec_off, bnd_off, gam_off;
  std::vector<int16_t> src_x, rec_x, bnd_x, gam_x;
  std::vector<int32_t> src_id, rec_id, gam_lin;
  int n_src = 0, n_rec = 0, n_bnd = 0, n_gam = 0;
};

bool in_pml(const fwi_params& p, int ix, int iy, int iz) {
  return ix < p.pml[0] || ix > p.nx - 1 - p.pml[0] || iy < p.pml[1] || iy > p.ny - 1 - p.pml[1] ||
         iz < p.pml[2] || iz > p.nz - 1 - p.pml[2];
}

int validate_params(const fwi_params* p) {
  if (!p) return fail(FWI_ERR_INVALID_ARG, "params is NULL");
  if (p->precision != 4 && p->precision != 8) return fail(FWI_ERR_INVALID_ARG, "precision must be 4 or 8");
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0 || (p->nx & 1)) return fail(FWI_ERR_INVALID_ARG, "bad grid size");
  if (!length_supported(p->nx / 2) || !length_supported(p->ny) || !length_supported(p->nz))
    return fail(FWI_ERR_UNSUPPORTED, "grid size not in the supported FFT set");
  if (p->nx / 2 > 32767) return fail(FWI_ERR_UNSUPPORTED, "nx too large");
  if (!(p->dx > 0) || !(p->dt > 0) || !(p->c_ref > 0) || !(p->rho0 > 0) || !(p->c_min > 0) ||
      !(p->c_max >= p->c_min) || !(p->pml_alpha >= 0))
    return fail(FWI_ERR_INVALID_ARG, "non-positive physical parameter");
  if (p->nt < 1) return fail(FWI_ERR_INVALID_ARG, "nt must be >= 1");
  if (p->batch < 1) return fail(FWI_ERR_INVALID_ARG, "batch must be >= 1");
  for (int a = 0; a < 3; ++a) {
    const int n = a == 0 ? p->nx : (a == 1 ? p->ny : p->nz);
    if (p->pml[a] < 0 || 2 * p->pml[a] >= n) return fail(FWI_ERR_INVALID_ARG, "PML thicker than the grid");
  }
  // kappa's series is evaluated for c_ref dt |k| / 2 <= pi / 2
  const double kmax2 = 3.0 * (kPi / p->dx) * (kPi / p->dx);
  const double u = (p->c_ref * p->dt / 2) * (p->c_ref * p->dt / 2) * kmax2;
  if (u > (kPi / 2) * (kPi / 2) * 1.0000001)
    return fail(FWI_ERR_INVALID_ARG, "c_ref dt too large for the k-space operator (c_ref dt sqrt(3) pi / dx > pi)");
  return FWI_OK;
}

int build_geometry(const fwi_params& p, const fwi_geometry* g, Geometry& out) {
  if (!g) return fail(FWI_ERR_INVALID_ARG, "geometry is NULL");
  if (g->n_src < 0 || g->n_rec < 0 || (g->n_src > 0 && !g->src_ijk) || (g->n_rec > 0 && !g->rec_ijk) ||
      !g->gamma_mask || !g->boundary_mask)
    return fail(FWI_ERR_INVALID_ARG, "geometry arrays missing");
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int nlines = ny * nz;
  out.nlines = nlines;
  const uint8_t* gm = g->gamma_mask;
  const uint8_t* bm = g->boundary_mask;
  auto lin = [&](int ix, int iy, int iz) { return ((size_t)iz * ny + iy) * nx + ix; };
  // transducers: per-line CSR, sorted by (line, x)
  auto build_list = [&](int n, const int32_t* ijk, std::vector<int32_t>& off, std::vector<int16_t>& xs,
                        std::vector<int32_t>& ids, const char* what) -> int {
    std::vector<std::pair<long long, int>> key(n);
    for (int i = 0; i < n; ++i) {
      const int ix = ijk[3 * i], iy = ijk[3 * i + 1], iz = ijk[3 * i + 2];
      if (ix < 0 || ix >= nx || iy < 0 || iy >= ny || iz < 0 || iz >= nz)
        return fail(FWI_ERR_INVALID_ARG, std::string(what) + " outside the grid");
      if (in_pml(p, ix, iy, iz)) return fail(FWI_ERR_INVALID_ARG, std::string(what) + " inside the PML");
      if (gm[lin(ix, iy, iz)]) return fail(FWI_ERR_INVALID_ARG, std::string(what) + " inside Gamma");
      key[i] = {(long long)lin(ix, iy, iz), i};
    }
    std::sort(key.begin(), key.end());
    for (int i = 1; i < n; ++i)
      if (key[i].first == key[i - 1].first) return fail(FWI_ERR_INVALID_ARG, std::string("duplicate ") + what + " voxel");
    off.assign(nlines + 1, 0);
    xs.resize(n);
    ids.resize(n);
    for (int i = 0; i < n; ++i) {
      const long long L = key[i].first;
      off[L / nx + 1]++;
      xs[i] = (int16_t)(L % nx);
      ids[i] = key[i].second;
    }
    for (int l = 0; l < nlines; ++l) off[l + 1] += off[l];
    return FWI_OK;
  };
  int rc = build_list(g->n_src, g->src_ijk, out.src_off, out.src_x, out.src_id, "source");
  if (rc) return rc;
  rc = build_list(g->n_rec, g->rec_ijk, out.rec_off, out.rec_x, out.rec_id, "receiver");
  if (rc) return rc;
  out.n_src = g->n_src;
  out.n_rec = g->n_rec;
  // Gamma and dGamma in line-major order
  out.gam_off.assign(nlines + 1, 0);
  out.bnd_off.assign(nlines + 1, 0);
  out.gam_x.clear();
  out.bnd_x.clear();
  out.gam_lin.clear();
  for (int line = 0; line < nlines; ++line) {
    const int iy = line % ny, iz = line / ny;
    for (int ix = 0; ix < nx; ++ix) {
      const size_t q = lin(ix, iy, iz);
      if (bm[q] && !gm[q]) return fail(FWI_ERR_INVALID_ARG, "dGamma voxel outside Gamma");
      if (gm[q]) {
        if (in_pml(p, ix, iy, iz)) return fail(FWI_ERR_INVALID_ARG, "Gamma touches the PML");
        out.gam_x.push_back((int16_t)ix);
        out.gam_lin.push_back((int32_t)q);
      }
      if (bm[q]) out.bnd_x.push_back((int16_t)ix);
    }
    out.gam_off[line + 1] = (int32_t)out.gam_x.size();
    out.bnd_off[line + 1] = (int32_t)out.bnd_x.size();
  }
  out.n_gam = (int)out.gam_x.size();
  out.n_bnd = (int)out.bnd_x.size();
  if ((long long)nx * ny * nz > 2147483647LL) return fail(FWI_ERR_UNSUPPORTED, "grid too large for int32 indices");
  return FWI_OK;
}

inline int spec_pitch(const fwi_params& p) {
  const int tw = p.precision == 4 ? pitch_tw<float>() : pitch_tw<double>();
  const int mh = p.nx / 2 + 1;
  return (mh + tw - 1) / tw * tw;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

struct Layout {
  size_t slots_bytes = 0;    // 2*batch slots
  size_t slot_bytes = 0;
  // offsets inside a slot: [v_x | V_y | V_z] [rho_x rho_y rho_z] [spec0 spec1 spec2]
  size_t vy_off = 0, vz_off = 0, vel_bytes = 0, rho_off = 0, spec_off = 0;
  size_t tape_bytes = 0;
  size_t traces_bytes = 0;   // internal traces
  size_t adj_bytes = 0;
  size_t ring_bytes = 0;
  size_t gacc_bytes = 0;
  size_t partial_bytes = 0;
  size_t tables_bytes = 0;
  size_t geom_bytes = 0;
  size_t delay_bytes = 0;    // [batch][n_src] int32 source delays
  size_t total = 0;
};

Layout make_layout(const fwi_params& p, const Geometry& g) {
  Layout L;
  const size_t rs = p.precision;
  const size_t nfield = (size_t)p.nx * p.ny * p.nz;
  const size_t nspec = (size_t)spec_pitch(p) * p.ny * p.nz;
  L.vy_off = align256(nfield * rs);
  L.vz_off = L.vy_off + align256(nspec * 2 * rs);
  L.vel_bytes = L.vz_off + align256(nspec * 2 * rs);
  L.rho_off = L.vel_bytes;
  L.spec_off = L.rho_off + align256(3 * nfield * rs);
  L.slot_bytes = L.spec_off + align256(3 * nspec * 2 * rs);
  L.slots_bytes = 2 * (size_t)p.batch * L.slot_bytes;
  L.tape_bytes = align256((size_t)p.batch * p.nt * std::max(g.n_bnd, 1) * rs);
  L.traces_bytes = align256((size_t)p.batch * p.nt * std::max(g.n_rec, 1) * rs);
  L.adj_bytes = L.traces_bytes;
  L.ring_bytes = align256((size_t)p.batch * 3 * std::max(g.n_gam, 1) * rs);
  L.gacc_bytes = align256((size_t)p.batch * std::max(g.n_gam, 1) * 8);
  const int nblk = (std::max(g.n_rec, 1) + 255) / 256;
  L.partial_bytes = align256((size_t)p.batch * nblk * 8);
  const int M = p.nx / 2;
  L.tables_bytes = align256(((size_t)M + p.ny + p.nz + (M + 1)) * 2 * rs) +
                   align256(((size_t)(M + 1) + p.ny + p.nz) * rs) +
                   align256(((size_t)(M + 1) + p.ny + p.nz) * 2 * 2 * rs) +
                   align256(((size_t)p.nx + p.ny + p.nz) * 2 * rs) + 4096;
  L.geom_bytes = align256(((size_t)g.nlines + 1) * 4 * 4) +
                 align256(((size_t)g.n_src + g.n_rec + g.n_bnd + g.n_gam) * 2) +
                 align256(((size_t)g.n_src + g.n_rec + g.n_gam) * 4) + 4096;
  L.delay_bytes = align256((size_t)p.batch * std::max(g.n_src, 1) * 4);
  L.total = L.slots_bytes + L.tape_bytes + L.traces_bytes + L.adj_bytes + L.ring_bytes + L.gacc_bytes +
            L.partial_bytes + L.tables_bytes + L.geom_bytes + L.delay_bytes + 256;
  return L;
}

// Device memory owned by a handle
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// Sampled HIP-event timing of pass launches (fwi_timing_enable / _read).
struct PassTimer {
  struct Pending {
    hipEvent_t a, b;
    int kind;
    double bytes;
  };
  int every = 0;
  bool active = false;   // sampling the current time step
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[FWI_PASS_COUNT] = {};
  double ms[FWI_PASS_COUNT] = {};
  double bytes[FWI_PASS_COUNT] = {};

  ~PassTimer() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void sample(int step) { active = every > 0 && (step % every) == 0; }
  hipEvent_t begin(hipStream_t st) {
    if (!active) return nullptr;
    hipEvent_t a = get();
    if (a) (void)hipEventRecord(a, st);
    return a;
  }
  void end(hipEvent_t a, int kind, double nbytes, hipStream_t st) {
    if (!a) return;
    hipEvent_t b = get();
    if (!b) { pool.push_back(a); return; }
    (void)hipEventRecord(b, st);
    pending.push_back({a, b, kind, nbytes});
  }
  hipError_t collect(hipStream_t st) {
    active = false;
    if (pending.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (auto& p : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        launches[p.kind] += 1;
        ms[p.kind] += t;
        bytes[p.kind] += p.bytes;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
    return hipSuccess;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// typed engine
// ---------------------------------------------------------------------------
struct EngineBase {
  virtual ~EngineBase() = default;
  virtual int forward(int B, const void* c, const void* src, const int8_t* w, void* traces, int flags,
                      hipStream_t st) = 0;
  virtual int gradient(int B, const void* c, const void* src, const int8_t* w, const void* obs, double* misfit,
                       void* grad, int flags, hipStream_t st) = 0;
  virtual int backward(int B, const void* c, const void* resid, double* misfit, void* grad, int flags,
                       hipStream_t st) = 0;
  virtual int derivative(const void* in, void* out, int axis, int sign, hipStream_t st) = 0;
  // power-law absorption (Sec. 2.1); alpha0 == 0 with no field switches it off
  virtual int set_absorption(double alpha0, double y, const void* field, int tr_flip) = 0;
  // whole-step source delays [B][n_src] (host), B = 0 switches them off
  virtual int set_delays(int B, const int32_t* host) = 0;
  // Gamma-compact vectors: compact[k] = full[gamma voxel k] (gather) or back
  virtual int gamma_copy(const void* src, void* dst, bool gather, hipStream_t st) = 0;
  virtual long long gamma_count() const = 0;
  // whole-grid 3D transform through the scratch slot's first spectrum:
  // forward = x R2C, y, z (unnormalised) of a real field; inverse = z, y, x C2R
  virtual int transform3d(const void* in, void* out, bool forward, hipStream_t st) = 0;
  virtual void* spectrum() = 0;
  virtual Dims dims() const = 0;
  virtual double spacing() const = 0;
  virtual int dev() const = 0;
  PassTimer timer;
  // axis-pass tile row segments in bytes (run-time tuning, fwi_set_tuning)
  int tile_bytes[3] = {FWI_Y_TILE_BYTES, FWI_ZM_TILE_BYTES, FWI_ZP_TILE_BYTES};
  // radix plans of the axis-pass kinds (AxisKind) and of the velocity and
  // density x passes (run-time tuning)
  int plans[3] = {FWI_Y_PLAN, FWI_ZM_PLAN, FWI_ZP_PLAN};
  int x_plan = FWI_X_PLAN;
};

template <typename T> struct Engine : EngineBase {
  using C = cplx<T>;
  fwi_params p{};
  Geometry geo;
  Layout lay;
  Dims d{};
  int device = 0;
  DevBuf mem_slots, mem_tape, mem_traces, mem_adj, mem_ring, mem_gacc, mem_partial, mem_tables, mem_geom,
      mem_slot_table, mem_flag, mem_delay;
  Tables<T> tb{};
  LineGeom lg{};
  Slot<T>* slot_table = nullptr;  // device [2*batch]
  std::vector<Slot<T>> slots_host;
  T* tape = nullptr;
  T* traces_int = nullptr;
  T* adj = nullptr;
  T* ring = nullptr;
  double* gacc = nullptr;
  double* partial = nullptr;
  int32_t* gam_lin = nullptr;
  int* flag = nullptr;
  int* step_counter = nullptr;   // device step index of replayed step graphs
  int32_t* delay = nullptr;      // [batch][n_src] whole-step source delays (eq. DelaySE)
  bool delays_on = false;
  bool mean_out = false;         // FWI_MEAN: one averaged gradient grid
  bool use_graph = false;
  int nblk_rec = 1;
  bool tape_valid = false;
  int tape_B = 0;
  T scale = 0, kap_a = 0;
  // absorption (set_absorption): the lossy passes replace X2 while set
  bool lossy = false;
  double a0u = 0.0, ypow = 1.5;
  const T* a0f = nullptr;
  bool tr_flip = true;
  DevBuf mem_padj;
  T* padj = nullptr;
  // A[d] spectrum per slot (the lossy Z1 writes it, Y2 and the lossy EOS read it)
  DevBuf mem_ad;
  C* ad_ptr = nullptr;
  // exact gradient (FWI_EXACT): dp/dc0 history on Gamma [nt][n_gam] and the
  // linear voxel index of every receiver (allocated on first use)
  DevBuf mem_hist, mem_rec_lin;
  T* hist_ptr = nullptr;          // non-null only during the forward of an exact gradient

  int init(const fwi_params& prm, Geometry&& g, int dev) {
    p = prm;
    geo = std::move(g);
    device = dev;
    lay = make_layout(p, geo);
    FWI_HIP(hipSetDevice(device));
    d.nx = p.nx; d.ny = p.ny; d.nz = p.nz; d.M = p.nx / 2; d.px = spec_pitch(p);
    d.nfield = (long long)p.nx * p.ny * p.nz;
    d.nspec = (long long)d.px * p.ny * p.nz;
    d.nlines = p.ny * p.nz;
    d.n_src = geo.n_src; d.n_rec = geo.n_rec; d.n_bnd = geo.n_bnd; d.n_gam = geo.n_gam;
    d.nt = p.nt;
    nblk_rec = (std::max(geo.n_rec, 1) + 255) / 256;
    auto alloc = [&](DevBuf& b, size_t n) -> int {
      if (hipMalloc(&b.p, std::max<size_t>(n, 256)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FWI_ERR_OOM, "device allocation of " + std::to_string(n) + " bytes failed");
      }
      return FWI_OK;
    };
    int rc;
    if ((rc = alloc(mem_slots, lay.slots_bytes))) return rc;
    if ((rc = alloc(mem_tape, lay.tape_bytes))) return rc;
    if ((rc = alloc(mem_traces, lay.traces_bytes))) return rc;
    if ((rc = alloc(mem_adj, lay.adj_bytes))) return rc;
    if ((rc = alloc(mem_ring, lay.ring_bytes))) return rc;
    if ((rc = alloc(mem_gacc, lay.gacc_bytes))) return rc;
    if ((rc = alloc(mem_partial, lay.partial_bytes))) return rc;
    if ((rc = alloc(mem_tables, lay.tables_bytes))) return rc;
    if ((rc = alloc(mem_geom, lay.geom_bytes))) return rc;
    if ((rc = alloc(mem_slot_table, sizeof(Slot<T>) * 2 * p.batch))) return rc;
    if ((rc = alloc(mem_flag, 256))) return rc;
    if ((rc = alloc(mem_delay, lay.delay_bytes))) return rc;
    delay = (int32_t*)mem_delay.p;
    tape = (T*)mem_tape.p;
    traces_int = (T*)mem_traces.p;
    adj = (T*)mem_adj.p;
    ring = (T*)mem_ring.p;
    gacc = (double*)mem_gacc.p;
    partial = (double*)mem_partial.p;
    flag = (int*)mem_flag.p;
    step_counter = flag + 16;
    // slots: [v_x | V_y | V_z | rho_x rho_y rho_z | spec0 spec1 spec2], 2*batch of
    // them; v_x is a real field, V_y and V_z are x spectra (rows of px complex)
    slots_host.resize(2 * p.batch);
    char* base = (char*)mem_slots.p;
    for (int s = 0; s < 2 * p.batch; ++s) {
      char* sb = base + (size_t)s * lay.slot_bytes;
      slots_host[s].v[0] = (T*)sb;
      slots_host[s].v[1] = (T*)(sb + lay.vy_off);
      slots_host[s].v[2] = (T*)(sb + lay.vz_off);
      T* r = (T*)(sb + lay.rho_off);
      for (int a = 0; a < 3; ++a) slots_host[s].rho[a] = r + (size_t)a * d.nfield;
      C* sp = (C*)(sb + lay.spec_off);
      for (int a = 0; a < 3; ++a) slots_host[s].spec[a] = sp + (size_t)a * d.nspec;
    }
    slot_table = (Slot<T>*)mem_slot_table.p;
    FWI_HIP(hipMemcpy(slot_table, slots_host.data(), sizeof(Slot<T>) * slots_host.size(), hipMemcpyHostToDevice));
    if ((rc = build_tables())) return rc;
    if ((rc = upload_geometry())) return rc;
    // clear the whole workspace once so that no uninitialised value is ever
    // read, on a private stream that is waited for alone: a handle created
    // while other handles compute does not wait for their work
    struct InitStream {
      hipStream_t s = nullptr;
      ~InitStream() {
        if (s) (void)hipStreamDestroy(s);
      }
    } init;
    FWI_HIP(hipStreamCreateWithFlags(&init.s, hipStreamNonBlocking));
    FWI_HIP(hipMemsetAsync(mem_slots.p, 0, lay.slots_bytes, init.s));
    FWI_HIP(hipMemsetAsync(mem_ring.p, 0, lay.ring_bytes, init.s));
    FWI_HIP(hipMemsetAsync(mem_delay.p, 0, lay.delay_bytes, init.s));
    FWI_HIP(hipStreamSynchronize(init.s));
    return FWI_OK;
  }

  int build_tables() {
    const int M = d.M, nx = p.nx, ny = p.ny, nz = p.nz;
    const double dx = p.dx;
    std::vector<C> h_tw_x(M), h_tw_y(ny), h_tw_z(nz), h_rtw(M + 1);
    auto W = [](long long m, long long n) {
      const double ang = -2.0 * kPi * (double)m / (double)n;
      C c;
      c.x = (T)std::cos(ang);
      c.y = (T)std::sin(ang);
      return c;
    };
    for (int m = 0; m < M; ++m) h_tw_x[m] = W(m, M);
    for (int m = 0; m < ny; ++m) h_tw_y[m] = W(m, ny);
    for (int m = 0; m < nz; ++m) h_tw_z[m] = W(m, nz);
    for (int k = 0; k <= M; ++k) h_rtw[k] = W(k, nx);
    // wavenumbers: x half spectrum k = 0..M, y / z signed (fftfreq)
    std::vector<double> kx(M + 1), ky(ny), kz(nz);
    for (int i = 0; i <= M; ++i) kx[i] = 2.0 * kPi * i / (nx * dx);
    for (int i = 0; i < ny; ++i) ky[i] = 2.0 * kPi * signed_freq(i, ny) / (ny * dx);
    for (int i = 0; i < nz; ++i) kz[i] = 2.0 * kPi * signed_freq(i, nz) / (nz * dx);
    const std::vector<double>* ks[3] = {&kx, &ky, &kz};
    std::vector<T> h_ksq[3];
    std::vector<C> h_sp[3], h_sm[3];
    for (int a = 0; a < 3; ++a) {
      const auto& k = *ks[a];
      h_ksq[a].resize(k.size());
      h_sp[a].resize(k.size());
      h_sm[a].resize(k.size());
      for (size_t i = 0; i < k.size(); ++i) {
        h_ksq[a][i] = (T)(k[i] * k[i]);
        // i k exp(+- i k dx / 2) = k (-sin(k dx/2), cos(k dx/2)) / k (sin, cos)
        const double h = k[i] * dx / 2.0;
        h_sp[a][i].x = (T)(-k[i] * std::sin(h));
        h_sp[a][i].y = (T)(k[i] * std::cos(h));
        h_sm[a][i].x = (T)(k[i] * std::sin(h));
        h_sm[a][i].y = (T)(k[i] * std::cos(h));
      }
    }
    const int lens[3] = {nx, ny, nz};
    std::vector<T> h_pn[3], h_ps[3];
    for (int a = 0; a < 3; ++a) {
      auto pn = pml_profile(lens[a], p.pml[a], dx, p.dt, p.c_ref, p.pml_alpha, false);
      auto ps = pml_profile(lens[a], p.pml[a], dx, p.dt, p.c_ref, p.pml_alpha, true);
      h_pn[a].assign(pn.begin(), pn.end());
      h_ps[a].assign(ps.begin(), ps.end());
    }
    scale = (T)(1.0 / ((double)nx * ny * nz));
    kap_a = (T)((p.c_ref * p.dt / 2.0) * (p.c_ref * p.dt / 2.0));
    // pack into the tables buffer
    char* base = (char*)mem_tables.p;
    size_t off = 0;
    auto put = [&](const void* src, size_t bytes) -> void* {
      void* dst = base + off;
      off += align256(bytes);
      return dst;
    };
    std::vector<std::pair<void*, std::pair<const void*, size_t>>> copies;
    auto place = [&](const void* src, size_t bytes) -> void* {
      void* dst = put(src, bytes);
      copies.push_back({dst, {src, bytes}});
      return dst;
    };
    tb.tw_x = (const C*)place(h_tw_x.data(), h_tw_x.size() * sizeof(C));
    tb.tw_y = (const C*)place(h_tw_y.data(), h_tw_y.size() * sizeof(C));
    tb.tw_z = (const C*)place(h_tw_z.data(), h_tw_z.size() * sizeof(C));
    tb.rtw = (const C*)place(h_rtw.data(), h_rtw.size() * sizeof(C));
    for (int a = 0; a < 3; ++a) {
      tb.ksq[a] = (const T*)place(h_ksq[a].data(), h_ksq[a].size() * sizeof(T));
      tb.sfac_p[a] = (const C*)place(h_sp[a].data(), h_sp[a].size() * sizeof(C));
      tb.sfac_m[a] = (const C*)place(h_sm[a].data(), h_sm[a].size() * sizeof(C));
      tb.pml_n[a] = (const T*)place(h_pn[a].data(), h_pn[a].size() * sizeof(T));
      tb.pml_s[a] = (const T*)place(h_ps[a].data(), h_ps[a].size() * sizeof(T));
    }
    if (off > lay.tables_bytes) return fail(FWI_ERR_HIP, "internal: table layout overflow");
    for (auto& c : copies) FWI_HIP(hipMemcpy(c.first, c.second.first, c.second.second, hipMemcpyHostToDevice));
    return FWI_OK;
  }

  int upload_geometry() {
    char* base = (char*)mem_geom.p;
    size_t off = 0;
    std::vector<std::pair<void*, std::pair<const void*, size_t>>> copies;
    auto place = [&](const void* src, size_t bytes) -> void* {
      void* dst = base + off;
      off += align256(std::max<size_t>(bytes, 4));
      if (bytes) copies.push_back({dst, {src, bytes}});
      return dst;
    };
    lg.src_off = (const int32_t*)place(geo.src_off.data(), geo.src_off.size() * 4);
    lg.rec_off = (const int32_t*)place(geo.rec_off.data(), geo.rec_off.size() * 4);
    lg.bnd_off = (const int32_t*)place(geo.bnd_off.data(), geo.bnd_off.size() * 4);
    lg.gam_off = (const int32_t*)place(geo.gam_off.data(), geo.gam_off.size() * 4);
    lg.src_x = (const int16_t*)place(geo.src_x.data(), geo.src_x.size() * 2);
    lg.rec_x = (const int16_t*)place(geo.rec_x.data(), geo.rec_x.size() * 2);
    lg.bnd_x = (const int16_t*)place(geo.bnd_x.data(), geo.bnd_x.size() * 2);
    lg.gam_x = (const int16_t*)place(geo.gam_x.data(), geo.gam_x.size() * 2);
    lg.src_id = (const int32_t*)place(geo.src_id.data(), geo.src_id.size() * 4);
    lg.rec_id = (const int32_t*)place(geo.rec_id.data(), geo.rec_id.size() * 4);
    gam_lin = (int32_t*)place(geo.gam_lin.data(), geo.gam_lin.size() * 4);
    if (off > lay.geom_bytes) return fail(FWI_ERR_HIP, "internal: geometry layout overflow");
    for (auto& c : copies) FWI_HIP(hipMemcpy(c.first, c.second.first, c.second.second, hipMemcpyHostToDevice));
    return FWI_OK;
  }

  // --- launch helpers -----------------------------------------------------
  AxisArgs<T> axis_args(int slot0, int na, int slot1, int nf, int f0) const {
    AxisArgs<T> a;
    a.slots = slot_table; a.slot0 = slot0; a.na = na; a.slot1 = slot1; a.nf = nf; a.f0 = f0;
    a.d = d; a.tb = tb; a.scale = scale; a.kap_a = kap_a;
    a.vcoef = (T)((double)p.nx * p.dt / p.rho0);
    a.half_e0 = (T)((ypow - 1.0) / 2.0);
    a.half_e1 = (T)((ypow - 2.0) / 2.0);
    a.vz_state = 0;
    for (int k = 0; k < 3; ++k) a.pml[k] = p.pml[k];
    a.ad = nullptr;
    a.ad_stride = d.nspec;
    a.ad_coef = (T)p.rho0;
    return a;
  }
  // tiles per spectrum row of an axis pass of kind k (AxisKind)
  int ntx(int k) const { return ntx_bytes(tile_bytes[k]); }
  int ntx_bytes(int tb) const {
    const int tw = tb / (int)sizeof(C);
    return (d.px + tw - 1) / tw;
  }
  // z passes of the absorption (the lossy Z1 with A[d], the fractional
  // Laplacian pass): 64-byte tiles whatever the Z1 tuning (at 448x448x224
  // FP32 the lossy gradient takes 14.4 s with them, 15.8 s with 128-byte ones)
  static constexpr int kLossyZTile = 64;

  // algorithmic bytes of one half spectrum / one real field
  double sbytes() const { return (double)(d.M + 1) * d.ny * d.nz * sizeof(C); }
  double fbytes() const { return (double)d.nfield * sizeof(T); }
  // fraction of the x-lines in a y or z PML slab: they keep the three split
  // densities and receive d-_y v_y and d-_z v_z apart; the others keep the
  // undamped sum (+ rho_x on the x-PML pairs) and receive d-_y v_y + d-_z v_z
  double full_line_frac() const {
    auto in = [](int i, int n, int P) { return i < P || i > n - 1 - P; };
    long long full = 0;
    for (int z = 0; z < d.nz; ++z)
      for (int y = 0; y < d.ny; ++y) full += (in(y, d.ny, p.pml[1]) || in(z, d.nz, p.pml[2])) ? 1 : 0;
    return (double)full / (double)d.nlines;
  }
  // split-density reads + writes of one density step, in fields: 6 on the
  // full lines, 2 plus rho_x on the x-PML pairs elsewhere (density_update)
  double rho_fields() const {
    auto in = [](int i, int n, int P) { return i < P || i > n - 1 - P; };
    long long xp = 0;
    for (int n = 0; n < d.M; ++n) xp += (in(2 * n, d.nx, p.pml[0]) || in(2 * n + 1, d.nx, p.pml[0])) ? 1 : 0;
    const double f = full_line_frac();
    return 6.0 * f + (2.0 + 4.0 * xp / d.nx) * (1.0 - f);
  }

  // Y3 .. Y2 of one step (six passes; X2 follows); half_only stops after the
  // velocity passes (Z2 with v_z, Y4 with v_y, X1 with v_x)
  int step_spectral(int slot0, int na, int slot1, int nslots, hipStream_t st, bool half_only = false) {
    const int ty = tile_bytes[AK_Y], tzm = tile_bytes[AK_ZMINUS], tzp = tile_bytes[AK_ZPLUS];
    const dim3 gy(ntx(AK_Y) * d.nz, nslots * 1);
    const dim3 gz(ntx(AK_ZPLUS) * d.ny, nslots), gz3(ntx(AK_ZMINUS) * d.ny, nslots * 3);
    const double S = sbytes(), F = fbytes(), ns = nslots;
    hipEvent_t ev;
    ev = timer.begin(st);
    FWI_HIP(launch_axis_y<T>(d.ny, false, ty, plans[AK_Y], gy, st, axis_args(slot0, na, slot1, 1, 0)));   // Y3
    timer.end(ev, FWI_PASS_Y_FWD, 2 * ns * S, st);
    ev = timer.begin(st);
    AxisArgs<T> az = axis_args(slot0, na, slot1, 1, 0);
    az.vz_state = 1;
    FWI_HIP(launch_axis_zp<T>(d.nz, tzp, plans[AK_ZPLUS], gz, st, az));        // Z2: Q, v_z
    timer.end(ev, FWI_PASS_Z_PLUS, 4 * ns * S, st);
    ev = timer.begin(st);
    FWI_HIP(launch_axis_yv<T>(d.ny, ty, plans[AK_Y], gy, st, axis_args(slot0, na, slot1, 1, 0)));    // Y4: Q, v_y
    timer.end(ev, FWI_PASS_Y_VEL_Q, 5 * ns * S, st);
    XArgs<T> xa;
    xa.slots = slot_table; xa.slot0 = slot0; xa.na = na; xa.slot1 = slot1;
    xa.d = d; xa.tb = tb; xa.dt_rho = (T)(p.dt / p.rho0);
    const int lpb = x_lines_per_block_vel<T>(d.M);
    ev = timer.begin(st);
    FWI_HIP(launch_x_vel<T>(d.M, x_plan, dim3((d.nlines + lpb - 1) / lpb, nslots), st, xa));   // X1 (v_x)
    timer.end(ev, FWI_PASS_X_VEL, ns * (2 * S + 2 * F), st);
    if (half_only) return FWI_OK;
    ev = timer.begin(st);
    FWI_HIP(launch_axis_y<T>(d.ny, false, ty, plans[AK_Y], gy, st, axis_args(slot0, na, slot1, 1, 0)));   // Y1 (v_x)
    timer.end(ev, FWI_PASS_Y_FWD, 2 * ns * S, st);
    ev = timer.begin(st);
    AxisArgs<T> a1 = axis_args(slot0, na, slot1, 3, 0);
    a1.vz_state = 1;
    if (lossy) {   // with A[d] of the absorption operator: one workgroup per tile and slot
      a1.ad = ad_ptr;
      FWI_HIP(launch_axis_zma<T>(d.nz, kLossyZTile, plans[AK_ZMINUS], dim3(ntx_bytes(kLossyZTile) * d.ny, nslots), st,
                                 a1));  // Z1 + A[d]
    } else {
      FWI_HIP(launch_axis_zm<T>(d.nz, tzm, plans[AK_ZMINUS], gz3, st, a1));  // Z1
    }
    timer.end(ev, FWI_PASS_Z_MINUS, (lossy ? 7 : 6) * ns * S, st);
    ev = timer.begin(st);
    const int thalf = tile_bytes[AK_Y] / (int)sizeof(C) / 2;   // columns per field of a paired tile
    const dim3 gy2(((lossy ? 2 : 1) * ntx(AK_Y) + (d.px + thalf - 1) / thalf) * d.nz, nslots);
    AxisArgs<T> a2 = axis_args(slot0, na, slot1, 3, 0);
    if (lossy) a2.ad = ad_ptr;
    FWI_HIP(launch_axis_yd<T>(d.ny, ty, plans[AK_Y], gy2, st, a2));   // Y2 (+ A[d])
    timer.end(ev, FWI_PASS_Y_INV, (5 + full_line_frac() + (lossy ? 2 : 0)) * ns * S, st);
    return FWI_OK;
  }

  X2Args<T> x2_args(int B, const T* c) const {
    X2Args<T> a{};
    a.slots = slot_table; a.B = B; a.tr_off = p.batch;
    a.d = d; a.tb = tb; a.g = lg;
    a.dt_rho0 = (T)(p.dt * p.rho0);
    a.src_k = (T)(2.0 * p.dt / (3.0 * p.dx));
    a.c = c;
    a.ring = ring; a.gacc = gacc;
    a.delay = delays_on ? delay : nullptr;
    a.hist = hist_ptr;
    for (int k = 0; k < 3; ++k) a.pml[k] = p.pml[k];
    a.ad = ad_ptr;
    a.ad_stride = d.nspec;
    return a;
  }
  int launch_x2(int mode, int B, const X2Args<T>& a, hipStream_t st) {
    const int lpb = x_lines_per_block_den<T>(d.M, mode);
    const double S = sbytes(), F = fbytes(), t = sizeof(T);
    hipEvent_t ev = (mode == XM_FWD || mode == XM_PAIR) ? timer.begin(st) : nullptr;
    FWI_HIP(launch_x_den<T>(d.M, mode, x_plan, dim3((d.nlines + lpb - 1) / lpb, B), st, a));
    if (mode == XM_FWD) {
      // 3 spectra in, 1 out, split densities r/w, c0, source row, trace row, tape row
      const double sp = 3 + full_line_frac();   // spectra read (the third on full lines only) and written
      const double b = B * (sp * S + (1 + rho_fields()) * F + t * (d.n_src + d.n_rec + (a.tape ? d.n_bnd : 0)));
      timer.end(ev, FWI_PASS_X_DEN_FWD, b, st);
    } else if (mode == XM_PAIR) {
      // two simulations of (4 S + split densities), c0 once, adjoint source
      // row, tape row, ring (2 reads + 1 write), FP64 accumulator read + write
      const double sp = 3 + full_line_frac();
      const double b = B * (2 * (sp * S + rho_fields() * F) + F + t * (d.n_rec + d.n_bnd + 3.0 * d.n_gam) + 16.0 * d.n_gam);
      timer.end(ev, FWI_PASS_X_DEN_PAIR, b, st);
    }
    return FWI_OK;
  }

  // --- lossy passes (absorption) -------------------------------------------
  void lossy_args(X2Args<T>& a) const {
    a.rho0 = (T)p.rho0;
    a.alpha0 = a0f;
    a.alpha0_u = (T)a0u;
    a.y1 = (T)(ypow - 1.0);
    a.two_tan = (T)(2.0 * std::tan(kPi * ypow / 2.0));
    a.tr_tau_sign = tr_flip ? (T)-1 : (T)1;
    a.padj = padj;
  }
  // density update, fractional Laplacians and equation of state of the
  // simulations of kind k0 (and k1 >= 0 in the same launches of the axis
  // passes): XL1, forward y, absorption z, inverse y, XL2
  int lossy_eos(int B, int k0, int k1, const X2Args<T>& a, hipStream_t st) {
    const int lpb = x_lines_per_block_den<T>(d.M);
    const dim3 gx((d.nlines + lpb - 1) / lpb, B);
    FWI_HIP(launch_x_lossy<T>(d.M, 0, k0, gx, st, a));
    if (k1 >= 0) FWI_HIP(launch_x_lossy<T>(d.M, 0, k1, gx, st, a));
    const int s0 = (k0 == SP_ADJOINT) ? 0 : p.batch;
    const int s1 = (k1 < 0) ? s0 : ((k1 == SP_ADJOINT) ? 0 : p.batch);
    const int ns = (k1 < 0) ? B : 2 * B;
    const int ty = tile_bytes[AK_Y], tz = kLossyZTile;
    // B[s] only: A[d] came with the step's Z1
    const AxisArgs<T> ax = axis_args(s0, B, s1, 1, 0);
    FWI_HIP(launch_axis_y<T>(d.ny, false, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, ns), st, ax));
    FWI_HIP(launch_axis_zf<T>(d.nz, tz, plans[AK_ZMINUS], dim3(ntx_bytes(tz) * d.ny, ns), st, ax));
    FWI_HIP(launch_axis_y<T>(d.ny, true, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, ns), st, ax));
    const int lpe = x_lines_per_block_eos<T>(d.M);
    const dim3 ge((d.nlines + lpe - 1) / lpe, B);
    FWI_HIP(launch_x_lossy<T>(d.M, 1, k0, ge, st, a));
    if (k1 >= 0) FWI_HIP(launch_x_lossy<T>(d.M, 1, k1, ge, st, a));
    return FWI_OK;
  }
  int lossy_grad(int B, const T* c, const X2Args<T>& a, bool adj_only, hipStream_t st) {
    if (d.n_gam == 0) return FWI_OK;
    const int blocks = (int)std::min<long long>((d.n_gam + 255) / 256, 4096);
    hipLaunchKernelGGL((k_lossy_grad<T>), dim3(blocks, B), dim3(256), 0, st, c, gam_lin, padj, ring, gacc,
                       (int)d.n_gam, (long long)d.nfield, a.ring_a, a.ring_b, a.ring_c, adj_only ? 1 : 0,
                       a.step_dev);
    FWI_HIP(hipGetLastError());
    return FWI_OK;
  }
  // Alg. 1 setup after the residual and the interleaved iterations, lossy:
  // the TR switches the sign of tau (unless tr_flip is off) and starts from
  // the tape only; gradient in the lossless form (2 / c0^3, ring of p_tr)
  int lossy_adjoint_tr(int B, const T* c, hipStream_t st) {
    const int N = p.nt, tr0 = p.batch;
    int rc;
    X2Args<T> a = x2_args(B, c);
    lossy_args(a);
    a.adj_src = adj; a.tape = tape;
    for (int b = 0; b < B; ++b)
      if ((rc = zero_velocity(tr0 + b, st))) return rc;
    a.tr_state_mode = 1; a.tape_row = N - 1; a.ring_c = 0; a.step = 0;
    if ((rc = lossy_eos(B, SP_DIRICHLET, -1, a, st))) return rc;
    a.tr_state_mode = 0;
    if (N == 1) {  // p_tr^(1) = 0 (ring slot 1; slot 0 holds p_tr^(0))
      if ((rc = zero_ring_slot(B, 1, st))) return rc;
    }
    if (N >= 2) {  // advance the TR by one step to get ahead of the adjoint
      if ((rc = step_spectral(tr0, B, tr0, B, st))) return rc;
      a.tape_row = N - 2; a.ring_c = 1;
      if ((rc = lossy_eos(B, SP_DIRICHLET, -1, a, st))) return rc;
    }
    int j0 = 0;
    if (use_graph && N >= 3) {   // iterations j = 0 .. N-3 pair with TR steps 2 .. N-1
      if ((rc = fill<int>(step_counter, 1, 0, st))) return rc;
      X2Args<T> ag = a;
      ag.step_dev = step_counter;
      if ((rc = replay_graph([&]() -> int {
             int r;
             if ((r = step_spectral(0, B, tr0, 2 * B, st))) return r;
             if ((r = lossy_eos(B, SP_ADJOINT, SP_DIRICHLET, ag, st))) return r;
             if ((r = lossy_grad(B, c, ag, false, st))) return r;
             return count_step(st);
           }, N - 2, st)))
        return rc;
      j0 = N - 2;
    }
    for (int j = j0; j < N; ++j) {
      const int k = j + 2;
      a.step = j;
      a.ring_a = j % 3; a.ring_b = (j + 1) % 3; a.ring_c = k % 3;
      if (k <= N - 1) {
        if ((rc = step_spectral(0, B, tr0, 2 * B, st))) return rc;
        a.tape_row = N - 1 - k;
        if ((rc = lossy_eos(B, SP_ADJOINT, SP_DIRICHLET, a, st))) return rc;
        if ((rc = lossy_grad(B, c, a, false, st))) return rc;
      } else {
        if ((rc = step_spectral(0, B, 0, B, st))) return rc;
        if ((rc = lossy_eos(B, SP_ADJOINT, -1, a, st))) return rc;
        if ((rc = lossy_grad(B, c, a, true, st))) return rc;
      }
    }
    return FWI_OK;
  }

  int set_absorption(double alpha0, double y, const void* field, int flip) override {
    if (!std::isfinite(alpha0) || alpha0 < 0.0) return fail(FWI_ERR_INVALID_ARG, "alpha0 must be finite and >= 0");
    if (alpha0 == 0.0 && !field) {
      tape_valid = false;
      lossy = false;
      a0f = nullptr;
      a0u = 0.0;
      return FWI_OK;
    }
    if (!(y > 0.0 && y < 2.0) || y == 1.0)
      return fail(FWI_ERR_INVALID_ARG, "power-law exponent y must lie in (0, 2) and differ from 1");
    if (!mem_padj.p) {
      FWI_HIP(hipSetDevice(device));
      const size_t n = std::max<size_t>((size_t)p.batch * std::max<long long>(d.n_gam, 1) * sizeof(T), 256);
      if (hipMalloc(&mem_padj.p, n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FWI_ERR_OOM, "device allocation of " + std::to_string(n) + " bytes failed");
      }
      padj = (T*)mem_padj.p;
    }
    if (!mem_ad.p) {
      FWI_HIP(hipSetDevice(device));
      const size_t n = (size_t)2 * p.batch * (size_t)d.nspec * sizeof(C);
      if (hipMalloc(&mem_ad.p, n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FWI_ERR_OOM, "device allocation of " + std::to_string(n) + " bytes failed");
      }
      ad_ptr = (C*)mem_ad.p;
    }
    tape_valid = false;
    lossy = true;
    a0u = alpha0;
    a0f = (const T*)field;
    ypow = y;
    tr_flip = flip != 0;
    return FWI_OK;
  }

  template <typename U> int fill(U* ptr, long long n, U v, hipStream_t st) {
    if (n <= 0) return FWI_OK;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((k_fill<U>), dim3(blocks), dim3(256), 0, st, ptr, n, v);
    FWI_HIP(hipGetLastError());
    return FWI_OK;
  }
  // zero the whole state (v, rho, spectra) of slots [s0, s0 + n)
  int zero_slots(int s0, int n, hipStream_t st) {
    char* b = (char*)mem_slots.p + (size_t)s0 * lay.slot_bytes;
    return fill<T>((T*)b, (long long)(n * lay.slot_bytes / sizeof(T)), (T)0, st);
  }
  // the velocity block of a slot: v_x, V_y, V_z (contiguous)
  long long vel_reals() const { return (long long)(lay.vel_bytes / sizeof(T)); }
  int zero_velocity(int s, hipStream_t st) { return fill<T>(slots_host[s].v[0], vel_reals(), (T)0, st); }

  int check_c(int B, const T* c, hipStream_t st) {
    FWI_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
    const long long n = (long long)B * d.nfield;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL((k_check_range<T>), dim3(blocks), dim3(256), 0, st, c, n, (T)p.c_min, (T)p.c_max, flag);
    FWI_HIP(hipGetLastError());
    int h = 0;
    FWI_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    FWI_HIP(hipStreamSynchronize(st));
    if (h) return fail(FWI_ERR_INVALID_ARG, "sound speed outside [c_min, c_max] or not finite");
    return FWI_OK;
  }
  int check_finite(const T* x, long long n, hipStream_t st) {
    FWI_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    const T big = (T)3.0e38;
    hipLaunchKernelGGL((k_check_range<T>), dim3(blocks), dim3(256), 0, st, x, n, -big, big, flag);
    FWI_HIP(hipGetLastError());
    int h = 0;
    FWI_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    FWI_HIP(hipStreamSynchronize(st));
    if (h) return fail(FWI_ERR_UNSTABLE, "non-finite value in the result");
    return FWI_OK;
  }

  // Capture body() (the launches of one time step) into a graph and replay
  // it `count` times on st.  The step counter must be set before.
  template <typename F> int replay_graph(F body, int count, hipStream_t st) {
    if (count <= 0) return FWI_OK;
    if (st == nullptr) return fail(FWI_ERR_INVALID_ARG, "FWI_GRAPH needs a non-null stream (capture)");
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    const bool was = timer.every > 0;
    const int every = timer.every;
    timer.every = 0;  // no event records inside a capture
    timer.active = false;
    FWI_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = body();
    hipError_t e = hipStreamEndCapture(st, &g);
    timer.every = was ? every : 0;
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(FWI_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(FWI_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < count && e == hipSuccess; ++i) e = hipGraphLaunch(ge, st);
    (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(FWI_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return FWI_OK;
  }
  int count_step(hipStream_t st) {
    hipLaunchKernelGGL(k_step_count, dim3(1), dim3(64), 0, st, step_counter);
    FWI_HIP(hipGetLastError());
    return FWI_OK;
  }

  // --- Alg. 1 forward iteration ------------------------------------------
  int run_forward(int B, const T* c, const T* src, const int8_t* w, T* traces, bool save, hipStream_t st) {
    const int tr0 = p.batch;
    int rc;
    if ((rc = zero_slots(tr0, B, st))) return rc;   // p^0 = 0, v = 0, rho = 0
    X2Args<T> a = x2_args(B, c);
    a.src_sig = src; a.w = w; a.traces = traces; a.tape = save ? tape : nullptr;
    if (lossy) {
      lossy_args(a);
      if (use_graph) {
        if ((rc = fill<int>(step_counter, 1, 0, st))) return rc;
        a.step_dev = step_counter;
        return replay_graph([&]() -> int {
          int r;
          if ((r = step_spectral(tr0, B, tr0, B, st))) return r;
          if ((r = lossy_eos(B, SP_SOURCE, -1, a, st))) return r;
          return count_step(st);
        }, p.nt, st);
      }
      for (int n = 0; n < p.nt; ++n) {
        if ((rc = step_spectral(tr0, B, tr0, B, st))) return rc;
        a.step = n;
        if ((rc = lossy_eos(B, SP_SOURCE, -1, a, st))) return rc;
      }
      return FWI_OK;
    }
    if (use_graph) {
      if ((rc = fill<int>(step_counter, 1, 0, st))) return rc;
      a.step_dev = step_counter;
      return replay_graph([&]() -> int {
        int r;
        if ((r = step_spectral(tr0, B, tr0, B, st))) return r;
        if ((r = launch_x2(XM_FWD, B, a, st))) return r;
        return count_step(st);
      }, p.nt, st);
    }
    for (int n = 0; n < p.nt; ++n) {
      timer.sample(n);
      if ((rc = step_spectral(tr0, B, tr0, B, st))) return rc;
      a.step = n;
      if ((rc = launch_x2(XM_FWD, B, a, st))) return rc;
    }
    return FWI_OK;
  }

  // --- Alg. 1 setup + interleaved adjoint / TR iterations ------------------
  int run_adjoint_tr(int B, const T* c, const T* resid_or_obs, bool is_resid, const T* fwd_traces,
                     double* misfit, T* grad, bool final_state, hipStream_t st) {
    const int N = p.nt, tr0 = p.batch;
    int rc;
    // residual, misfit, reversed running sum (the adjoint source)
    hipLaunchKernelGGL((k_residual<T>), dim3(nblk_rec, B), dim3(256), 0, st, fwd_traces, resid_or_obs,
                       is_resid ? 1 : 0, adj, partial, N, d.n_rec);
    FWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_misfit_final, dim3((B + 63) / 64), dim3(64), 0, st, partial, nblk_rec, misfit, B);
    FWI_HIP(hipGetLastError());
    if ((rc = fill<double>(gacc, (long long)B * d.n_gam, 0.0, st))) return rc;
    if ((rc = zero_slots(0, B, st))) return rc;           // adjoint state
    if (lossy) {
      if (final_state) return fail(FWI_ERR_INVALID_ARG, "FWI_TR_FINAL_STATE is not available with absorption");
      if ((rc = lossy_adjoint_tr(B, c, st))) return rc;
      return scatter_grad(B, grad, st);
    }
    X2Args<T> a = x2_args(B, c);
    a.adj_src = adj; a.tape = tape;
    // TR initial state: zero interior (or the final forward state), dGamma <- g^{N-1}
    if (final_state) {
      // the forward slots still hold v^{N-1/2}, rho^N and the x-spectrum of
      // p^N: one more velocity update gives v^{N+1/2}; the TR starts from
      // (rho^N, -v^{N+1/2}) so that its first velocity update returns -v^{N-1/2}
      if ((rc = step_spectral(tr0, B, tr0, B, st, true))) return rc;
      for (int b = 0; b < B; ++b) {
        hipLaunchKernelGGL((k_scale<T>), dim3(4096), dim3(256), 0, st, slots_host[tr0 + b].v[0],
                           vel_reals(), (T)-1);
        FWI_HIP(hipGetLastError());
      }
      a.tr_state_mode = 2;
    } else {
      for (int b = 0; b < B; ++b)
        if ((rc = zero_velocity(tr0 + b, st))) return rc;
      a.tr_state_mode = 1;
    }
    a.tape_row = N - 1; a.ring_c = 0; a.step = 0;
    if ((rc = launch_x2(XM_TRONLY, B, a, st))) return rc;
    a.tr_state_mode = 0;
    if (N == 1) {  // p_tr^(1) = 0 (ring slot 1; slot 0 holds p_tr^(0))
      if ((rc = zero_ring_slot(B, 1, st))) return rc;
    }
    if (N >= 2) {  // advance the TR by one step to get ahead of the adjoint
      if ((rc = step_spectral(tr0, B, tr0, B, st))) return rc;
      a.tape_row = N - 2; a.ring_c = 1;
      if ((rc = launch_x2(XM_TRONLY, B, a, st))) return rc;
    }
    int j0 = 0;
    if (use_graph && N >= 3) {   // iterations j = 0 .. N-3 pair with TR steps 2 .. N-1
      if ((rc = fill<int>(step_counter, 1, 0, st))) return rc;
      X2Args<T> ag = a;
      ag.step_dev = step_counter;
      if ((rc = replay_graph([&]() -> int {
             int r;
             if ((r = step_spectral(0, B, tr0, 2 * B, st))) return r;
             if ((r = launch_x2(XM_PAIR, B, ag, st))) return r;
             return count_step(st);
           }, N - 2, st)))
        return rc;
      j0 = N - 2;
    }
    for (int j = j0; j < N; ++j) {
      const int k = j + 2;
      timer.sample(j);
      a.step = j;
      a.ring_a = j % 3; a.ring_b = (j + 1) % 3; a.ring_c = k % 3;
      if (k <= N - 1) {
        if ((rc = step_spectral(0, B, tr0, 2 * B, st))) return rc;
        a.tape_row = N - 1 - k;
        if ((rc = launch_x2(XM_PAIR, B, a, st))) return rc;
      } else {
        if ((rc = step_spectral(0, B, 0, B, st))) return rc;
        if ((rc = launch_x2(XM_ADJONLY, B, a, st))) return rc;
      }
    }
    timer.active = false;
    return scatter_grad(B, grad, st);
  }
  int zero_ring_slot(int B, int slot, hipStream_t st) {
    int rc;
    for (int b = 0; b < B; ++b)
      if ((rc = fill<T>(ring + ((size_t)b * 3 + slot) * d.n_gam, (long long)d.n_gam, (T)0, st))) return rc;
    return FWI_OK;
  }
  // G on Gamma -> full grid, zero elsewhere ([B] grids, or their mean in one
  // grid when mean_out is set)
  int scatter_grad(int B, T* grad, hipStream_t st) {
    int rc;
    if (mean_out) {
      if ((rc = fill<T>(grad, (long long)d.nfield, (T)0, st))) return rc;
      if (d.n_gam > 0) {
        hipLaunchKernelGGL((k_grad_mean_scatter<T>), dim3((d.n_gam + 255) / 256), dim3(256), 0, st, gacc, gam_lin,
                           d.n_gam, grad, B);
        FWI_HIP(hipGetLastError());
      }
      return FWI_OK;
    }
    if ((rc = fill<T>(grad, (long long)B * d.nfield, (T)0, st))) return rc;
    if (d.n_gam > 0) {
      hipLaunchKernelGGL((k_grad_scatter<T>), dim3((d.n_gam + 255) / 256, B), dim3(256), 0, st, gacc, gam_lin,
                         d.n_gam, d.nfield, grad, B);
      FWI_HIP(hipGetLastError());
    }
    return FWI_OK;
  }

  int set_delays(int B, const int32_t* host) override {
    if (B < 0 || B > p.batch) return fail(FWI_ERR_INVALID_ARG, "B outside [0, batch]");
    if (B > 0 && !host) return fail(FWI_ERR_INVALID_ARG, "NULL delay array");
    std::vector<int32_t> rows((size_t)p.batch * std::max(d.n_src, 1), 0);
    for (long long i = 0; i < (long long)B * d.n_src; ++i) {
      if (host[i] < 0 || host[i] >= p.nt) return fail(FWI_ERR_INVALID_ARG, "delay outside [0, nt)");
      rows[i] = host[i];
    }
    FWI_HIP(hipSetDevice(device));
    FWI_HIP(hipDeviceSynchronize());   // no call of this handle may be reading the table
    FWI_HIP(hipMemcpy(delay, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    delays_on = B > 0;
    return FWI_OK;
  }

  int check_B(int B) {
    if (B < 1 || B > p.batch) return fail(FWI_ERR_INVALID_ARG, "B outside [1, batch]");
    return FWI_OK;
  }

  int forward(int B, const void* c, const void* src, const int8_t* w, void* traces, int flags,
              hipStream_t st) override {
    int rc;
    if ((rc = check_B(B))) return rc;
    if (!c || !traces || (d.n_src > 0 && (!src || !w))) return fail(FWI_ERR_INVALID_ARG, "NULL array argument");
    FWI_HIP(hipSetDevice(device));
    if (flags & FWI_CHECK_INPUT)
      if ((rc = check_c(B, (const T*)c, st))) return rc;
    const bool save = (flags & FWI_SAVE_TAPE) != 0;
    use_graph = (flags & FWI_GRAPH) != 0;
    tape_valid = false;
    if ((rc = run_forward(B, (const T*)c, (const T*)src, w, (T*)traces, save, st))) return rc;
    if (save) { tape_valid = true; tape_B = B; }
    FWI_HIP(timer.collect(st));
    if (flags & FWI_CHECK_FINITE)
      if ((rc = check_finite((const T*)traces, (long long)B * p.nt * d.n_rec, st))) return rc;
    return FWI_OK;
  }

  // Fractional Laplacians of two real fields in one set of passes (the
  // passes of the lossy equation of state): outB = B[inB] = F^-1 |k|^{y-1} F
  // inB, outA = A[inA] = F^-1 |k|^{y-2} F inA (both 0 at k = 0).  Uses the
  // spectra of the first forward slot.
  int frac_pair(const T* inB, const T* inA, T* outB, T* outA, hipStream_t st) {
    const int s = p.batch;
    XArgs<T> xa;
    xa.slots = slot_table; xa.slot0 = s; xa.na = 1; xa.slot1 = s;
    xa.d = d; xa.tb = tb; xa.dt_rho = (T)0;
    const int lpb = x_lines_per_block<T>(d.M);
    const dim3 gx((d.nlines + lpb - 1) / lpb, 1);
    const int ty = tile_bytes[AK_Y], tz = kLossyZTile;
    const AxisArgs<T> ax = axis_args(s, 1, s, 2, 0);
    FWI_HIP(launch_x_r2c<T>(d.M, gx, st, xa, inB, 0));
    FWI_HIP(launch_x_r2c<T>(d.M, gx, st, xa, inA, 1));
    FWI_HIP(launch_axis_y<T>(d.ny, false, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, 2), st, ax));
    FWI_HIP(launch_axis_zf<T>(d.nz, tz, plans[AK_ZMINUS], dim3(ntx_bytes(tz) * d.ny, 2), st, ax));
    FWI_HIP(launch_axis_y<T>(d.ny, true, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, 2), st, ax));
    FWI_HIP(launch_x_c2r<T>(d.M, gx, st, xa, outB, 0, nullptr));
    FWI_HIP(launch_x_c2r<T>(d.M, gx, st, xa, outA, 1, nullptr));
    return FWI_OK;
  }

  // The exact discrete gradient of D (FWI_EXACT): the forward iteration with
  // dp/dc0 at a fixed state stored on Gamma for every step, then reverse-mode
  // differentiation of every operation of the iteration, backwards in time:
  //   pb += M^T r^n;  G += pb * dp/dc0 (step n)
  //   sb = c0^2 pb - B[eta c0^2 pb],  db = A[tau c0^2 pb]       (absorption)
  //   rb_a += sb; t = L_a rb_a; rb_a = L_a t; vb_a -= d+_a (rho0 db - dt rho0 t)
  //   t = Ls_a vb_a; vb_a = Ls_a t; pb = dt/rho0 sum_a d-_a t
  // (d-^T = -d+, d+^T = -d-: the staggered multipliers are conjugate).  The
  // c0 of the source scaling is held fixed (as in the oracle).  Problem 0 only.
  int run_exact(const T* c, const T* src, const int8_t* w, const T* obs, bool is_resid, double* misfit, T* grad,
                hipStream_t st) {
    const int N = p.nt;
    int rc;
    if (!mem_hist.p) {
      const size_t n = std::max<size_t>((size_t)N * std::max<long long>(d.n_gam, 1) * sizeof(T), 256);
      if (hipMalloc(&mem_hist.p, n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FWI_ERR_OOM, "device allocation of " + std::to_string(n) + " bytes failed");
      }
    }
    if (!mem_rec_lin.p) {
      std::vector<int32_t> lin(std::max(d.n_rec, 1), 0);
      for (int line = 0; line < d.nlines; ++line)
        for (int i = geo.rec_off[line]; i < geo.rec_off[line + 1]; ++i)
          lin[geo.rec_id[i]] = line * d.nx + geo.rec_x[i];
      if (hipMalloc(&mem_rec_lin.p, lin.size() * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FWI_ERR_OOM, "receiver index allocation failed");
      }
      FWI_HIP(hipMemcpy(mem_rec_lin.p, lin.data(), lin.size() * 4, hipMemcpyHostToDevice));
    }
    T* hist = (T*)mem_hist.p;
    const int32_t* rec_lin = (const int32_t*)mem_rec_lin.p;
    // forward with the dp/dc0 history
    hist_ptr = hist;
    rc = run_forward(1, c, src, w, traces_int, false, st);
    hist_ptr = nullptr;
    if (rc) return rc;
    // misfit (the reversed running sum the kernel also writes is not used here)
    hipLaunchKernelGGL((k_residual<T>), dim3(nblk_rec, 1), dim3(256), 0, st, traces_int, obs, is_resid ? 1 : 0, adj,
                       partial, N, d.n_rec);
    FWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_misfit_final, dim3(1), dim3(64), 0, st, partial, nblk_rec, misfit, 1);
    FWI_HIP(hipGetLastError());
    // work fields: the adjoint slot and the real fields of the first forward
    // slot (its spectra are the transforms' scratch)
    const Slot<T>& s0 = slots_host[0];
    const Slot<T>& sS = slots_host[p.batch];
    T* vb[3] = {s0.rho[0], s0.rho[1], s0.rho[2]};
    T* rb[3] = {s0.v[0], s0.v[1], s0.v[2]};
    T* pb = (T*)s0.spec[0];
    T* FB = (T*)s0.spec[1];
    T* FA = (T*)s0.spec[2];
    T* eP = sS.rho[0];
    T* tP = sS.rho[1];
    T* ub = sS.rho[2];
    T* tmp = sS.v[0];
    T* tv = sS.v[1];
    const long long nf = d.nfield;
    for (int a = 0; a < 3; ++a) {
      if ((rc = fill<T>(vb[a], nf, (T)0, st))) return rc;
      if ((rc = fill<T>(rb[a], nf, (T)0, st))) return rc;
    }
    if ((rc = fill<T>(pb, nf, (T)0, st))) return rc;
    if ((rc = fill<double>(gacc, d.n_gam, 0.0, st))) return rc;
    const int nb = (int)std::min<long long>((nf + 255) / 256, 16384);
    const int gb = (int)std::max<long long>(1, std::min<long long>((d.n_gam + 255) / 256, 8192));
    const T dt_rho0 = (T)(p.dt * p.rho0), rho0 = (T)p.rho0, dt_over_rho0 = (T)(p.dt / p.rho0);
    for (int n = N - 1; n >= 0; --n) {
      hipLaunchKernelGGL((k_ex_inject<T>), dim3((d.n_rec + 255) / 256 + 1), dim3(256), 0, st, pb, rec_lin,
                         traces_int, obs, is_resid ? 1 : 0, n, d.n_rec);
      FWI_HIP(hipGetLastError());
      if (d.n_gam > 0) {
        hipLaunchKernelGGL((k_ex_accum<T>), dim3(gb), dim3(256), 0, st, gacc, pb, gam_lin,
                           hist + (size_t)n * d.n_gam, (int)d.n_gam);
        FWI_HIP(hipGetLastError());
      }
      if (lossy) {
        hipLaunchKernelGGL((k_ex_coef<T>), dim3(nb), dim3(256), 0, st, c, a0f, (T)a0u, ypow,
                           2.0 * std::tan(kPi * ypow / 2.0), pb, eP, tP, nf);
        FWI_HIP(hipGetLastError());
        if ((rc = frac_pair(eP, tP, FB, FA, st))) return rc;
      }
      for (int a = 0; a < 3; ++a) {
        hipLaunchKernelGGL((k_ex_rho<T>), dim3(nb), dim3(256), 0, st, c, pb, lossy ? FB : nullptr,
                           lossy ? FA : nullptr, rb[a], ub, tb.pml_n[a], a, d, dt_rho0, rho0);
        FWI_HIP(hipGetLastError());
        if ((rc = derivative(ub, tmp, a, +1, st))) return rc;
        hipLaunchKernelGGL((k_axpby<T>), dim3(nb), dim3(256), 0, st, nf, (T)-1, (const T*)tmp, (T)1, vb[a]);
        FWI_HIP(hipGetLastError());
      }
      if ((rc = fill<T>(pb, nf, (T)0, st))) return rc;
      for (int a = 0; a < 3; ++a) {
        hipLaunchKernelGGL((k_ex_vel<T>), dim3(nb), dim3(256), 0, st, vb[a], tv, tb.pml_s[a], a, d);
        FWI_HIP(hipGetLastError());
        if ((rc = derivative(tv, tmp, a, -1, st))) return rc;
        hipLaunchKernelGGL((k_axpby<T>), dim3(nb), dim3(256), 0, st, nf, dt_over_rho0, (const T*)tmp, (T)1, pb);
        FWI_HIP(hipGetLastError());
      }
    }
    return scatter_grad(1, grad, st);
  }

  int gradient(int B, const void* c, const void* src, const int8_t* w, const void* obs, double* misfit,
               void* grad, int flags, hipStream_t st) override {
    int rc;
    if ((rc = check_B(B))) return rc;
    if (!c || !obs || !misfit || !grad || (d.n_src > 0 && (!src || !w)))
      return fail(FWI_ERR_INVALID_ARG, "NULL array argument");
    FWI_HIP(hipSetDevice(device));
    if (flags & FWI_CHECK_INPUT)
      if ((rc = check_c(B, (const T*)c, st))) return rc;
    tape_valid = false;
    use_graph = (flags & FWI_GRAPH) != 0;
    mean_out = (flags & FWI_MEAN) != 0;
    if (flags & FWI_EXACT) {
      if (B != 1 || (flags & (FWI_GRAPH | FWI_MEAN | FWI_TR_FINAL_STATE)))
        return fail(FWI_ERR_INVALID_ARG, "FWI_EXACT takes B = 1 without FWI_GRAPH, FWI_MEAN, FWI_TR_FINAL_STATE");
      mean_out = false;
      if ((rc = run_exact((const T*)c, (const T*)src, w, (const T*)obs, false, misfit, (T*)grad, st))) return rc;
      FWI_HIP(timer.collect(st));
      if (flags & FWI_CHECK_FINITE)
        if ((rc = check_finite((const T*)grad, d.nfield, st))) return rc;
      return FWI_OK;
    }
    if ((rc = run_forward(B, (const T*)c, (const T*)src, w, traces_int, true, st))) return rc;
    if ((rc = run_adjoint_tr(B, (const T*)c, (const T*)obs, false, traces_int, misfit, (T*)grad,
                             (flags & FWI_TR_FINAL_STATE) != 0, st)))
      return rc;
    FWI_HIP(timer.collect(st));
    if (flags & FWI_CHECK_FINITE)
      if ((rc = check_finite((const T*)grad, (long long)(mean_out ? 1 : B) * d.nfield, st))) return rc;
    return FWI_OK;
  }

  int backward(int B, const void* c, const void* resid, double* misfit, void* grad, int flags,
               hipStream_t st) override {
    int rc;
    if ((rc = check_B(B))) return rc;
    if (!c || !resid || !misfit || !grad) return fail(FWI_ERR_INVALID_ARG, "NULL array argument");
    if (!tape_valid || tape_B != B) return fail(FWI_ERR_NO_TAPE, "no saved tape for this batch size");
    FWI_HIP(hipSetDevice(device));
    use_graph = (flags & FWI_GRAPH) != 0;
    mean_out = (flags & FWI_MEAN) != 0;
    if ((rc = run_adjoint_tr(B, (const T*)c, (const T*)resid, true, (const T*)resid, misfit, (T*)grad,
                             (flags & FWI_TR_FINAL_STATE) != 0, st)))
      return rc;
    FWI_HIP(timer.collect(st));
    if (flags & FWI_CHECK_FINITE)
      if ((rc = check_finite((const T*)grad, (long long)(mean_out ? 1 : B) * d.nfield, st))) return rc;
    return FWI_OK;
  }

  int gamma_copy(const void* src, void* dst, bool gather, hipStream_t st) override {
    if (!src || !dst) return fail(FWI_ERR_INVALID_ARG, "NULL vector");
    FWI_HIP(hipSetDevice(device));
    const long long n = d.n_gam;
    if (n == 0) return FWI_OK;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    if (gather) hipLaunchKernelGGL((k_gather<T>), dim3(blocks), dim3(256), 0, st, (const T*)src, gam_lin, n, (T*)dst);
    else hipLaunchKernelGGL((k_scatter<T>), dim3(blocks), dim3(256), 0, st, (const T*)src, gam_lin, n, (T*)dst);
    FWI_HIP(hipGetLastError());
    return FWI_OK;
  }
  long long gamma_count() const override { return d.n_gam; }

  int transform3d(const void* in, void* out, bool forward, hipStream_t st) override {
    FWI_HIP(hipSetDevice(device));
    const int s = p.batch;   // scratch: the first forward slot
    tape_valid = false;
    XArgs<T> xa;
    xa.slots = slot_table; xa.slot0 = s; xa.na = 1; xa.slot1 = s;
    xa.d = d; xa.tb = tb; xa.dt_rho = (T)0;
    const int lpb = x_lines_per_block<T>(d.M);
    const dim3 gx((d.nlines + lpb - 1) / lpb, 1);
    const int ty = tile_bytes[AK_Y], tz = tile_bytes[AK_ZMINUS];
    if (forward) {
      if (!in) return fail(FWI_ERR_INVALID_ARG, "NULL field");
      FWI_HIP(launch_x_r2c<T>(d.M, gx, st, xa, (const T*)in, 0));
      FWI_HIP(launch_axis_y<T>(d.ny, false, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, 1), st, axis_args(s, 1, s, 1, 0)));
      FWI_HIP(launch_axis_z<T>(d.nz, false, tz, plans[AK_ZMINUS], dim3(ntx(AK_ZMINUS) * d.ny, 1), st, axis_args(s, 1, s, 1, 0)));
    } else {
      if (!out) return fail(FWI_ERR_INVALID_ARG, "NULL field");
      FWI_HIP(launch_axis_z<T>(d.nz, true, tz, plans[AK_ZMINUS], dim3(ntx(AK_ZMINUS) * d.ny, 1), st, axis_args(s, 1, s, 1, 0)));
      FWI_HIP(launch_axis_y<T>(d.ny, true, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, 1), st, axis_args(s, 1, s, 1, 0)));
      FWI_HIP(launch_x_c2r<T>(d.M, gx, st, xa, (T*)out, 0, nullptr));
    }
    return FWI_OK;
  }
  void* spectrum() override { return slots_host[p.batch].spec[0]; }
  Dims dims() const override { return d; }
  double spacing() const override { return p.dx; }
  int dev() const override { return device; }

  int derivative(const void* in, void* out, int axis, int sign, hipStream_t st) override {
    if (!in || !out || axis < 0 || axis > 2 || (sign != 1 && sign != -1))
      return fail(FWI_ERR_INVALID_ARG, "bad derivative arguments");
    FWI_HIP(hipSetDevice(device));
    const int s = p.batch;   // scratch: the first forward slot
    tape_valid = false;
    XArgs<T> xa;
    xa.slots = slot_table; xa.slot0 = s; xa.na = 1; xa.slot1 = s;
    xa.d = d; xa.tb = tb; xa.dt_rho = (T)0;
    const int lpb = x_lines_per_block<T>(d.M);
    const dim3 gx((d.nlines + lpb - 1) / lpb, 1);
    const int f = sign > 0 ? 0 : axis;
    FWI_HIP(launch_x_r2c<T>(d.M, gx, st, xa, (const T*)in, f));
    const int ty = tile_bytes[AK_Y], tzm = tile_bytes[AK_ZMINUS], tzp = tile_bytes[AK_ZPLUS];
    FWI_HIP(launch_axis_y<T>(d.ny, false, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, 1), st, axis_args(s, 1, s, 1, f)));
    if (sign > 0) {
      // Z2 and the split inverse y pass of the time step; the x shift factor
      // of d+_x is applied by the C2R
      FWI_HIP(launch_axis_zp<T>(d.nz, tzp, plans[AK_ZPLUS], dim3(ntx(AK_ZPLUS) * d.ny, 1), st, axis_args(s, 1, s, 1, 0)));
      FWI_HIP(launch_axis_ys<T>(d.ny, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, 2), st, axis_args(s, 1, s, 2, 0)));
    } else {
      FWI_HIP(launch_axis_zm<T>(d.nz, tzm, plans[AK_ZMINUS], dim3(ntx(AK_ZMINUS) * d.ny, 1), st, axis_args(s, 1, s, 1, axis)));
      FWI_HIP(launch_axis_y<T>(d.ny, true, ty, plans[AK_Y], dim3(ntx(AK_Y) * d.nz, 1), st, axis_args(s, 1, s, 1, axis)));
    }
    FWI_HIP(launch_x_c2r<T>(d.M, gx, st, xa, (T*)out, axis, (sign > 0 && axis == 0) ? tb.sfac_p[0] : nullptr));
    return FWI_OK;
  }
};

struct fwi_handle {
  std::unique_ptr<EngineBase> eng;
  int precision = 4;
};

// L-BFGS history on the device (Alg. 2 buffers S, Y): a ring of m pairs,
// rho_j = 1 / y_j^T s_j and the alpha_j of the last two-loop recursion.
struct fwi_lbfgs {
  int precision = 4, device = 0, m = 0;
  long long n = 0;
  void* S = nullptr;        // [m][n]
  void* Y = nullptr;        // [m][n]
  double* sc = nullptr;     // rho[m], alpha[m], coef, part[RED_BLOCKS]
  int count = 0, head = 0;  // stored pairs; ring slot of the oldest
  double* rho() const { return sc; }
  double* alpha() const { return sc + m; }
  double* coef() const { return sc + 2 * m; }
  double* part() const { return sc + 2 * m + 1; }
  char* vec(void* base, int slot) const { return (char*)base + (size_t)slot * n * precision; }
};

namespace {

int vec_blocks(long long n) { return (int)std::min<long long>((n + 255) / 256, 8192); }

// Scratch of one two-loop recursion: alpha[m], the coefficient of the second
// loop and the dot-product partial sums (part[RED_BLOCKS]).  fwi_lbfgs_apply
// takes it from the history's own allocation, fwi_lbfgs_apply_noalloc from
// the library's static device array.
struct LbfgsScratch {
  double* alpha;
  double* coef;
  double* part;
};

template <typename T>
int lbfgs_dot(fwi_lbfgs* L, double* part, const void* a, const void* b, int mode, const double* rho,
              const double* alpha, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_dot_partial<T>), dim3(RED_BLOCKS), dim3(RED_NT), 0, st, (const T*)a, (const T*)b, L->n,
                     part);
  FWI_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(RED_NT), 0, st, part, RED_BLOCKS, mode, rho, alpha, out);
  FWI_HIP(hipGetLastError());
  return FWI_OK;
}

template <typename T> int lbfgs_push(fwi_lbfgs* L, const void* s, const void* y, hipStream_t st) {
  int slot;
  if (L->count < L->m) {
    slot = (L->head + L->count) % L->m;
    L->count++;
  } else {
    slot = L->head;
    L->head = (L->head + 1) % L->m;
  }
  const size_t bytes = (size_t)L->n * sizeof(T);
  FWI_HIP(hipMemcpyAsync(L->vec(L->S, slot), s, bytes, hipMemcpyDeviceToDevice, st));
  FWI_HIP(hipMemcpyAsync(L->vec(L->Y, slot), y, bytes, hipMemcpyDeviceToDevice, st));
  return lbfgs_dot<T>(L, L->part(), L->vec(L->Y, slot), L->vec(L->S, slot), 1, nullptr, nullptr, L->rho() + slot,
                     st);
}

template <typename T>
int lbfgs_apply(fwi_lbfgs* L, const LbfgsScratch& w, const void* g, void* r, double h0, hipStream_t st) {
  const size_t bytes = (size_t)L->n * sizeof(T);
  if (g != r) FWI_HIP(hipMemcpyAsync(r, g, bytes, hipMemcpyDeviceToDevice, st));
  const int nb = vec_blocks(L->n);
  int rc;
  for (int j = L->count - 1; j >= 0; --j) {   // newest to oldest: alpha_j = rho_j s_j^T q, q -= alpha_j y_j
    const int slot = (L->head + j) % L->m;
    if ((rc = lbfgs_dot<T>(L, w.part, L->vec(L->S, slot), r, 2, L->rho() + slot, nullptr, w.alpha + slot, st)))
      return rc;
    hipLaunchKernelGGL((k_axpy_dev<T>), dim3(nb), dim3(256), 0, st, (T*)r, (const T*)L->vec(L->Y, slot),
                       w.alpha + slot, -1.0, L->n);
    FWI_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL((k_axpby<T>), dim3(nb), dim3(256), 0, st, L->n, (T)0, (const T*)nullptr, (T)h0, (T*)r);
  FWI_HIP(hipGetLastError());
  for (int j = 0; j < L->count; ++j) {        // oldest to newest: r += (alpha_j - rho_j y_j^T r) s_j
    const int slot = (L->head + j) % L->m;
    if ((rc = lbfgs_dot<T>(L, w.part, L->vec(L->Y, slot), r, 3, L->rho() + slot, w.alpha + slot, w.coef, st)))
      return rc;
    hipLaunchKernelGGL((k_axpy_dev<T>), dim3(nb), dim3(256), 0, st, (T*)r, (const T*)L->vec(L->S, slot), w.coef,
                       1.0, L->n);
    FWI_HIP(hipGetLastError());
  }
  return FWI_OK;
}

bool prec_ok(int p) { return p == 4 || p == 8; }

}  // namespace

// Static scratch of fwi_lbfgs_apply_noalloc: alpha[FWI_NOALLOC_MAX_PAIRS], the
// second-loop coefficient (padded to 8 doubles) and the RED_BLOCKS partial
// sums of each dot product.  Every device holds its own copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returned on that device (noalloc_scratch), never
// through the array's name.  Every value is written before it is read within
// one call, so nothing needs clearing between calls.
constexpr int kNoallocCoefOff = FWI_NOALLOC_MAX_PAIRS;
constexpr int kNoallocPartOff = FWI_NOALLOC_MAX_PAIRS + 8;
static __device__ __align__(256) double scratch[kNoallocPartOff + RED_BLOCKS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device` (resolved once per device with that
// device current, then cached).  Leaves `device` current.
int noalloc_scratch(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return fail(FWI_ERR_INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    FWI_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    FWI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(FWI_ERR_HIP, "hipGetSymbolAddress returned a null address for the static scratch");
    g_scratch_dev[device] = (double*)ptr;
  }
  *out = g_scratch_dev[device];
  return FWI_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

int fwi_create(const fwi_params* params, const fwi_geometry* geom, int device, fwi_handle** out) {
  if (!out) return fail(FWI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate_params(params);
  if (rc) return rc;
  Geometry g;
  if ((rc = build_geometry(*params, geom, g))) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return fail(FWI_ERR_HIP, "no such HIP device");
  }
  std::unique_ptr<fwi_handle> h(new fwi_handle());
  h->precision = params->precision;
  if (params->precision == 4) {
    auto e = std::make_unique<Engine<float>>();
    if ((rc = e->init(*params, std::move(g), device))) return rc;
    h->eng = std::move(e);
  } else {
    auto e = std::make_unique<Engine<double>>();
    if ((rc = e->init(*params, std::move(g), device))) return rc;
    h->eng = std::move(e);
  }
  *out = h.release();
  return FWI_OK;
}

void fwi_destroy(fwi_handle* h) { delete h; }

int64_t fwi_workspace_bytes(const fwi_params* params, const fwi_geometry* geom) {
  if (validate_params(params)) return 0;
  Geometry g;
  if (build_geometry(*params, geom, g)) return 0;
  Layout L = make_layout(*params, g);
  return (int64_t)(L.total + sizeof(Slot<double>) * 2 * params->batch + 256);
}

int fwi_rademacher(uint64_t seed, int32_t n, int8_t* w_out) {
  if (n < 0 || (n > 0 && !w_out)) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  // SplitMix64 (Steele, Lea, Flood 2014): golden-ratio increment, Stafford
  // variant-13 finaliser; output i uses state seed + (i + 1) * increment.
  for (int32_t i = 0; i < n; ++i) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    w_out[i] = (z >> 63) ? (int8_t)-1 : (int8_t)1;
  }
  return FWI_OK;
}

int fwi_delays(uint64_t seed, int32_t n, int32_t tau_steps, int32_t* out) {
  if (n < 0 || tau_steps < 0 || (n > 0 && !out)) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  for (int32_t i = 0; i < n; ++i) {
    uint64_t z = seed + (uint64_t)(n + i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    const double d = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    out[i] = (int32_t)std::floor(d * tau_steps + 0.5);
  }
  return FWI_OK;
}

int fwi_forward(fwi_handle* h, int32_t B, const void* c, const void* src_sig, const int8_t* w, void* traces,
                int32_t flags, fwi_stream_t stream) {
  if (!h) return fail(FWI_ERR_INVALID_ARG, "handle is NULL");
  return h->eng->forward(B, c, src_sig, w, traces, flags, (hipStream_t)stream);
}

int fwi_gradient(fwi_handle* h, int32_t B, const void* c, const void* src_sig, const int8_t* w, const void* obs,
                 double* misfit, void* grad, int32_t flags, fwi_stream_t stream) {
  if (!h) return fail(FWI_ERR_INVALID_ARG, "handle is NULL");
  return h->eng->gradient(B, c, src_sig, w, obs, misfit, grad, flags, (hipStream_t)stream);
}

int fwi_backward(fwi_handle* h, int32_t B, const void* c, const void* residual, double* misfit, void* grad,
                 int32_t flags, fwi_stream_t stream) {
  if (!h) return fail(FWI_ERR_INVALID_ARG, "handle is NULL");
  return h->eng->backward(B, c, residual, misfit, grad, flags, (hipStream_t)stream);
}

int fwi_derivative(fwi_handle* h, const void* in, void* out, int32_t axis, int32_t sign, fwi_stream_t stream) {
  if (!h) return fail(FWI_ERR_INVALID_ARG, "handle is NULL");
  return h->eng->derivative(in, out, axis, sign, (hipStream_t)stream);
}

int fwi_set_absorption(fwi_handle* h, double alpha0, double y, const void* alpha0_field, int32_t tr_flip) {
  if (!h) return fail(FWI_ERR_INVALID_ARG, "handle is NULL");
  return h->eng->set_absorption(alpha0, y, alpha0_field, tr_flip);
}

int fwi_set_delays(fwi_handle* h, int32_t B, const int32_t* delays) {
  if (!h) return fail(FWI_ERR_INVALID_ARG, "NULL handle");
  return h->eng->set_delays(B, delays);
}

int fwi_get_tuning(const fwi_handle* h, fwi_tuning* out) {
  if (!h || !out) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  out->y_tile_bytes = h->eng->tile_bytes[AK_Y];
  out->zm_tile_bytes = h->eng->tile_bytes[AK_ZMINUS];
  out->zp_tile_bytes = h->eng->tile_bytes[AK_ZPLUS];
  out->y_plan = h->eng->plans[AK_Y];
  out->zm_plan = h->eng->plans[AK_ZMINUS];
  out->zp_plan = h->eng->plans[AK_ZPLUS];
  out->x_plan = h->eng->x_plan;
  return FWI_OK;
}

int fwi_set_tuning(fwi_handle* h, const fwi_tuning* t) {
  if (!h || !t) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  const int v[3] = {t->y_tile_bytes, t->zm_tile_bytes, t->zp_tile_bytes};
  for (int k = 0; k < 3; ++k)
    if (v[k] != 64 && v[k] != 128) return fail(FWI_ERR_INVALID_ARG, "tile bytes must be 64 or 128");
  const int pl[4] = {t->y_plan, t->zm_plan, t->zp_plan, t->x_plan};
  for (int k = 0; k < 4; ++k)
    if (pl[k] != 0 && pl[k] != 1) return fail(FWI_ERR_INVALID_ARG, "radix plans must be 0 or 1");
  for (int k = 0; k < 3; ++k) {
    h->eng->tile_bytes[k] = v[k];
    h->eng->plans[k] = pl[k];
  }
  h->eng->x_plan = pl[3];
  return FWI_OK;
}

int fwi_timing_enable(fwi_handle* h, int32_t every) {
  if (!h || every < 0) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  h->eng->timer.every = every;
  return FWI_OK;
}

int fwi_timing_read(fwi_handle* h, int32_t pass, int64_t* launches, double* total_ms, double* total_bytes) {
  if (!h || pass < 0 || pass >= FWI_PASS_COUNT || !launches || !total_ms || !total_bytes)
    return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  PassTimer& t = h->eng->timer;
  *launches = t.launches[pass];
  *total_ms = t.ms[pass];
  *total_bytes = t.bytes[pass];
  t.launches[pass] = 0;
  t.ms[pass] = 0;
  t.bytes[pass] = 0;
  return FWI_OK;
}

int fwi_gamma_size(const fwi_handle* h, int64_t* n) {
  if (!h || !n) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  *n = h->eng->gamma_count();
  return FWI_OK;
}

int fwi_gamma_gather(fwi_handle* h, const void* full, void* compact, fwi_stream_t stream) {
  if (!h) return fail(FWI_ERR_INVALID_ARG, "handle is NULL");
  return h->eng->gamma_copy(full, compact, true, (hipStream_t)stream);
}

int fwi_gamma_scatter(fwi_handle* h, const void* compact, void* full, fwi_stream_t stream) {
  if (!h) return fail(FWI_ERR_INVALID_ARG, "handle is NULL");
  return h->eng->gamma_copy(compact, full, false, (hipStream_t)stream);
}

int fwi_interp_fourier(fwi_handle* coarse, fwi_handle* fine, const void* in, void* out, int32_t window,
                       fwi_stream_t stream) {
  if (!coarse || !fine || !in || !out || (window != 0 && window != 1))
    return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  if (coarse->precision != fine->precision) return fail(FWI_ERR_INVALID_ARG, "precisions differ");
  EngineBase& ec = *coarse->eng;
  EngineBase& ef = *fine->eng;
  if (ec.dev() != ef.dev()) return fail(FWI_ERR_INVALID_ARG, "handles on different devices");
  const Dims dc = ec.dims(), df = ef.dims();
  if (dc.nx > df.nx || dc.ny > df.ny || dc.nz > df.nz) return fail(FWI_ERR_INVALID_ARG, "fine grid smaller");
  const double lc[3] = {dc.nx * ec.spacing(), dc.ny * ec.spacing(), dc.nz * ec.spacing()};
  const double lf[3] = {df.nx * ef.spacing(), df.ny * ef.spacing(), df.nz * ef.spacing()};
  for (int a = 0; a < 3; ++a)
    if (std::fabs(lc[a] - lf[a]) > 1e-9 * lf[a]) return fail(FWI_ERR_INVALID_ARG, "grids cover different boxes");
  const hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = ec.transform3d(in, nullptr, true, st))) return rc;
  FWI_HIP(hipSetDevice(ef.dev()));
  const long long nf = (long long)df.px * df.ny * df.nz;
  const double scale = 1.0 / ((double)dc.nx * dc.ny * dc.nz);
  const int blocks = (int)std::min<long long>((nf + 255) / 256, 16384);
  if (fine->precision == 4)
    hipLaunchKernelGGL((k_spec_embed<float>), dim3(blocks), dim3(256), 0, st, (const cplx<float>*)ec.spectrum(), dc,
                       (cplx<float>*)ef.spectrum(), df, window, scale);
  else
    hipLaunchKernelGGL((k_spec_embed<double>), dim3(blocks), dim3(256), 0, st, (const cplx<double>*)ec.spectrum(),
                       dc, (cplx<double>*)ef.spectrum(), df, window, scale);
  FWI_HIP(hipGetLastError());
  return ef.transform3d(nullptr, out, false, st);
}

int fwi_resample_time(int32_t nt_in, int32_t n_ch, const void* in, double dt_in, int32_t nt_out, double dt_out,
                      double f_cut, double beta, double t_window, double scale, void* out, int32_t precision,
                      fwi_stream_t stream) {
  if (nt_in <= 0 || n_ch <= 0 || nt_out <= 0 || !in || !out || !(dt_in > 0) || !(dt_out > 0) || !(f_cut > 0) ||
      !(beta >= 0) || !(t_window > 0) || !prec_ok(precision))
    return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  const hipStream_t st = (hipStream_t)stream;
  const long long n = (long long)nt_out * n_ch;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 16384);
  if (precision == 4)
    hipLaunchKernelGGL((k_resample_time<float>), dim3(blocks), dim3(256), 0, st, (const float*)in, nt_in, n_ch, dt_in,
                       (float*)out, nt_out, dt_out, f_cut, beta, t_window, scale);
  else
    hipLaunchKernelGGL((k_resample_time<double>), dim3(blocks), dim3(256), 0, st, (const double*)in, nt_in, n_ch,
                       dt_in, (double*)out, nt_out, dt_out, f_cut, beta, t_window, scale);
  FWI_HIP(hipGetLastError());
  return FWI_OK;
}

int fwi_lbfgs_create(int64_t n, int32_t m, int32_t precision, int32_t device, fwi_lbfgs** out) {
  if (!out) return fail(FWI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n <= 0 || m <= 0 || !prec_ok(precision)) return fail(FWI_ERR_INVALID_ARG, "bad L-BFGS sizes");
  std::unique_ptr<fwi_lbfgs> L(new fwi_lbfgs());
  L->precision = precision; L->device = device; L->m = m; L->n = n;
  FWI_HIP(hipSetDevice(device));
  double* scratch_ptr = nullptr;   // resolve the static scratch of fwi_lbfgs_apply_noalloc on this device
  int rc = noalloc_scratch(device, &scratch_ptr);
  if (rc) return rc;
  const size_t vb = (size_t)m * n * precision;
  if (hipMalloc(&L->S, vb) != hipSuccess || hipMalloc(&L->Y, vb) != hipSuccess ||
      hipMalloc((void**)&L->sc, (2 * (size_t)m + 1 + RED_BLOCKS) * sizeof(double)) != hipSuccess) {
    if (L->S) (void)hipFree(L->S);
    if (L->Y) (void)hipFree(L->Y);
    if (L->sc) (void)hipFree(L->sc);
    return fail(FWI_ERR_OOM, "L-BFGS history allocation failed");
  }
  *out = L.release();
  return FWI_OK;
}

void fwi_lbfgs_destroy(fwi_lbfgs* L) {
  if (!L) return;
  (void)hipSetDevice(L->device);
  (void)hipFree(L->S);
  (void)hipFree(L->Y);
  (void)hipFree(L->sc);
  delete L;
}

int fwi_lbfgs_push(fwi_lbfgs* L, const void* s, const void* y, fwi_stream_t stream) {
  if (!L || !s || !y) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  FWI_HIP(hipSetDevice(L->device));
  return L->precision == 4 ? lbfgs_push<float>(L, s, y, (hipStream_t)stream)
                           : lbfgs_push<double>(L, s, y, (hipStream_t)stream);
}

int fwi_lbfgs_apply(fwi_lbfgs* L, const void* g, void* r, double h0, fwi_stream_t stream) {
  if (!L || !g || !r) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  FWI_HIP(hipSetDevice(L->device));
  const LbfgsScratch w{L->alpha(), L->coef(), L->part()};
  return L->precision == 4 ? lbfgs_apply<float>(L, w, g, r, h0, (hipStream_t)stream)
                           : lbfgs_apply<double>(L, w, g, r, h0, (hipStream_t)stream);
}

int fwi_lbfgs_apply_noalloc(fwi_lbfgs* L, const void* g, void* r, double h0, fwi_stream_t stream) {
  if (!L || !g || !r) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  if (L->m > FWI_NOALLOC_MAX_PAIRS)
    return fail(FWI_ERR_INVALID_ARG, "history of " + std::to_string(L->m) + " pairs exceeds the " +
                                         std::to_string((int)FWI_NOALLOC_MAX_PAIRS) +
                                         " pairs of fwi_lbfgs_apply_noalloc's static scratch");
  double* sp = nullptr;
  const int rc = noalloc_scratch(L->device, &sp);   // leaves L->device current
  if (rc) return rc;
  const LbfgsScratch w{sp, sp + kNoallocCoefOff, sp + kNoallocPartOff};
  return L->precision == 4 ? lbfgs_apply<float>(L, w, g, r, h0, (hipStream_t)stream)
                           : lbfgs_apply<double>(L, w, g, r, h0, (hipStream_t)stream);
}

int fwi_lbfgs_count(const fwi_lbfgs* L, int32_t* count) {
  if (!L || !count) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  *count = L->count;
  return FWI_OK;
}

int fwi_vec_axpby(int64_t n, double a, const void* x, double b, void* y, int32_t precision, fwi_stream_t stream) {
  if (n < 0 || !y || !prec_ok(precision)) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  if (n == 0) return FWI_OK;
  const hipStream_t st = (hipStream_t)stream;
  if (precision == 4)
    hipLaunchKernelGGL((k_axpby<float>), dim3(vec_blocks(n)), dim3(256), 0, st, (long long)n, (float)a,
                       (const float*)x, (float)b, (float*)y);
  else
    hipLaunchKernelGGL((k_axpby<double>), dim3(vec_blocks(n)), dim3(256), 0, st, (long long)n, a, (const double*)x, b,
                       (double*)y);
  FWI_HIP(hipGetLastError());
  return FWI_OK;
}

int fwi_vec_clip(int64_t n, void* x, double lo, double hi, int32_t precision, fwi_stream_t stream) {
  if (n < 0 || !x || !prec_ok(precision) || !(lo <= hi)) return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  if (n == 0) return FWI_OK;
  const hipStream_t st = (hipStream_t)stream;
  if (precision == 4)
    hipLaunchKernelGGL((k_clip<float>), dim3(vec_blocks(n)), dim3(256), 0, st, (long long)n, (float*)x, (float)lo,
                       (float)hi);
  else
    hipLaunchKernelGGL((k_clip<double>), dim3(vec_blocks(n)), dim3(256), 0, st, (long long)n, (double*)x, lo, hi);
  FWI_HIP(hipGetLastError());
  return FWI_OK;
}

int fwi_vec_sqslowness(int64_t n, int32_t mode, const void* in, const void* aux, void* out, int32_t precision,
                       fwi_stream_t stream) {
  if (n < 0 || !in || !out || mode < 0 || mode > 2 || (mode == 2 && !aux) || !prec_ok(precision))
    return fail(FWI_ERR_INVALID_ARG, "bad arguments");
  if (n == 0) return FWI_OK;
  const hipStream_t st = (hipStream_t)stream;
  if (precision == 4)
    hipLaunchKernelGGL((k_sqslowness<float>), dim3(vec_blocks(n)), dim3(256), 0, st, (long long)n, mode,
                       (const float*)in, (const float*)aux, (float*)out);
  else
    hipLaunchKernelGGL((k_sqslowness<double>), dim3(vec_blocks(n)), dim3(256), 0, st, (long long)n, mode,
                       (const double*)in, (const double*)aux, (double*)out);
  FWI_HIP(hipGetLastError());
  return FWI_OK;
}

const char* fwi_status_string(int status) {
  switch (status) {
    case FWI_OK: return "ok";
    case FWI_ERR_INVALID_ARG: return "invalid argument";
    case FWI_ERR_UNSUPPORTED: return "unsupported size";
    case FWI_ERR_OOM: return "out of device memory";
    case FWI_ERR_NO_TAPE: return "no saved tape";
    case FWI_ERR_HIP: return "HIP runtime error";
    case FWI_ERR_UNSTABLE: return "non-finite result";
    default: return "unknown status";
  }
}

const char* fwi_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
