// C ABI of the HIP Hubbard-response library: validation, device layout of the
// ground state, the self-consistent Sternheimer driver (FP64, or FP32/BF16 inner
// solves with FP64 residual refinement), CG iterations captured as hipGraphs, the
// launch-shape autotuner, and the assembly of chi0 / chi / U,V.  See include/hp.h for
// the contract of each entry point.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <string>
#include <algorithm>
#include <thread>
#include <vector>

#include <mutex>

#include "hp_internal.h"

using namespace hp;

// Fixed workspace of hp_apply_h_noalloc: the intermediate buffers of its operator apply
// live here, so that the call allocates nothing.  One copy per GPU the library runs on, held
// until the process ends.  In host code `scratch` is only a handle: its device address on
// each device comes from hipGetSymbolAddress (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[HP_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err = "no error";

hp_status fail(hp_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HPCHK(expr)                                                                          \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(e_ == hipErrorOutOfMemory ? HP_ERR_OOM : HP_ERR_HIP, "%s failed: %s (%s:%d)", #expr, \
                  hipGetErrorString(e_), __FILE__, __LINE__);                                \
  } while (0)

#define HPTRY(expr)                     \
  do {                                  \
    hp_status s_ = (expr);              \
    if (s_ < 0) return s_;              \
  } while (0)

// Radices in decimation-in-frequency order: at each step the first of 8, 9, 4, 2, 3, 5
// that divides (the device code derives the same sequence at compile time).
bool factor_235(int n, std::vector<int> &rad) {
  rad.clear();
  if (n < 1) return false;
  while (n > 1) {
    int r = 0;
    for (int c : {8, 9, 4, 2, 3, 5})
      if (n % c == 0) {
        r = c;
        break;
      }
    if (r == 0) return false;
    rad.push_back(r);
    n /= r;
  }
  return rad.size() <= 8;
}

// Position p of a decimation-in-frequency output holds natural index perm[p].
std::vector<int> dif_perm(int n, const std::vector<int> &rad) {
  std::vector<int> span, perm(n);
  int pr = 1;
  for (int r : rad) { pr *= r; span.push_back(n / pr); }
  for (int k = 0; k < n; ++k) {
    int kk = k, p = 0;
    for (size_t s = 0; s < rad.size(); ++s) { p += (kk % rad[s]) * span[s]; kk /= rad[s]; }
    perm[p] = k;
  }
  return perm;
}

template <class T>
hp_status dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? HP_ERR_OOM : HP_ERR_HIP, "hipMalloc of %zu bytes: %s",
                                   count * sizeof(T), hipGetErrorString(e));
  return HP_OK;
}

int wrapi(long v, int n) { long r = v % n; return (int)(r < 0 ? r + n : r); }

// Device address of `scratch` on the current device, looked up once per device.
hp_status noalloc_scratch(unsigned char **out) {
  static std::mutex mu;
  static std::vector<unsigned char *> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HP_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HP_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    addr[dev] = static_cast<unsigned char *>(ptr);
  }
  *out = addr[dev];
  return HP_OK;
}

struct HostEntry {
  std::array<double, 3> k;
  double weight;
  int npw;
  int spin = 0;
  std::vector<int> order;  // internal position -> caller index
  int pw_off = 0;          // offset of this entry in the per-plane-wave device arrays
};

}  // namespace

struct hp_ctx {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n1 = 0, n2 = 0, n3 = 0;
  long nr = 0, np = 0;
  int n_occ = 0, n_beta = 0, n_hub = 0, n_mesh = 0, n_kpts = 0;
  int n_kb = 0;  // KB rows among the n_beta rows of the stacked table (the rest carry V_Hub)
  // Spin: nspin blocks of entries.  Internally the mesh entries of every spin come first
  // (entry = spin * n_mesh_spin + k for mesh k), so that n_mesh = nspin * n_mesh_spin pairs
  // form one batch; internal_of maps a caller entry index to the internal one.
  int nspin = 1, n_mesh_spin = 0;
  double occ = 2.0;  // electrons per state
  std::vector<int> internal_of;
  std::vector<double> ent_eps;  // [n_kpts][n_occ] band energies of every entry (internal order)
  int ld = 0, ns_pad = 0, ns_max = 0, max_chunk_pw = 0, npw_max = 0, n_proj = 0;
  double cell[9], bvec[9], omega = 0, alpha = 0;
  std::vector<double> hub_tau;  // [n_hub][3] site positions (bohr)
  // metallic ground state (cold smearing of width degauss): per entry and kept band the
  // occupation f and the smearing delta d; per (site, q) the projection weights beta and the
  // row occupations on the device; the Fermi-level density and occupations for q = 0
  double degauss = 0.0, efermi = 0.0;
  std::vector<double> occ_f, occ_d;
  double *d_beta = nullptr, *d_focc = nullptr;
  double2 *d_rhoF = nullptr;
  std::vector<std::complex<double>> n_fermi;
  bool metal_q0 = false;     // the current right-hand sides are at q = 0 (Fermi-level shift)
  // of the current right-hand sides; complex because the response is linear over the
  // complex numbers (the response-potential iterates are complex)
  std::complex<double> fermi_shift = 0.0;
  std::vector<HostEntry> ent;
  std::vector<int> px, py;
  Plane pl{};
  Axis az{};
  Sticks sk{};
  // device allocations (freed by hp_destroy)
  std::vector<void *> allocs;
  double2 *tw = nullptr;
  int *d_px = nullptr, *d_py = nullptr;
  double *d_vp = nullptr, *d_fxc = nullptr, *d_bvec = nullptr, *d_q = nullptr;
  int *d_npw = nullptr;
  int *d_order = nullptr;  // [pw] internal position -> caller index, per entry at pw_off
  // this device's fixed workspace of hp_apply_h_noalloc (the file-scope `scratch` array)
  unsigned char *scratch = nullptr;
  double *d_kin = nullptr, *d_diag = nullptr, *d_rowscale = nullptr, *d_eps = nullptr;
  double2 *d_T = nullptr, *d_phi = nullptr, *d_A = nullptr, *d_psi = nullptr;
  KPair *d_kp = nullptr, *d_kself = nullptr;
  // work
  double2 *B = nullptr, *X = nullptr, *R = nullptr, *P = nullptr, *AP = nullptr;
  double2 *S1 = nullptr, *S2 = nullptr, *Cpart = nullptr, *C = nullptr, *Cphi = nullptr;
  double *rz = nullptr, *bn = nullptr, *rn = nullptr;
  int *active = nullptr, *count = nullptr;
  int *bmap = nullptr;  // [n_mesh][n_occ + 1] active bands of each pair, packed (GEMM tiles)
  double2 *part = nullptr, *drho = nullptr, *dvin = nullptr, *dvout = nullptr, *f = nullptr, *tmp = nullptr;
  double2 *fprev = nullptr, *dvprev = nullptr, *hdf = nullptr, *hdv = nullptr;
  double2 *dots_part = nullptr, *dots = nullptr, *dn = nullptr, *coef = nullptr;
  const double2 **ptrs = nullptr;
  // FP32 copies and work buffers of the mixed-precision inner solves (allocated on first use)
  bool have32 = false;
  float2 *tw32 = nullptr, *T32 = nullptr;
  unsigned *T16 = nullptr;  // the stacked table in packed bfloat16 (allocated on first use)
  float2 *psi32 = nullptr, *dv32 = nullptr;  // FP32 occupied states on the grid, response potential
  int lowp_gemm = 0;        // hp_scf_params.lowp_gemm of the current call
  float *vp32 = nullptr;
  float2 *X32 = nullptr, *R32 = nullptr, *B32 = nullptr, *P32 = nullptr, *AP32 = nullptr;
  // FP64 A X of the mixed solves' refinement residuals.  ax_valid: it holds A X for the
  // current X (the last solve ended on an FP64 residual); the next warm start of the same
  // operator then reuses it instead of applying A again.  Cleared by every solve that
  // does not end that way.
  double2 *AX = nullptr;
  bool ax_valid = false;
  double *bn_in = nullptr, *rn_in = nullptr, *rz_in = nullptr, *floor_in = nullptr;
  int *act_in = nullptr, *act_out = nullptr;
  Plane pl32{};
  Axis az32{};
  int nsplit_cap = 16;
  int drho_split = 1;
  long t_stride = 0, phi_stride = 0;
  hipEvent_t ev[16];
  // per-kernel timing (hp_profile_start / hp_profile_stop)
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  struct Pending {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  long prof_calls[32] = {0};
  double prof_ms[32] = {0};
  // CG iterations captured as hipGraphs: one executable graph per (operator precision,
  // iterations per launch, profiling on/off, batch).  Every kernel of a captured iteration
  // reads its tolerance and writes its counters through the fixed device pointers below.
  struct CgGraph {
    int kind, len, prof, nk, lowp, tuned;
    const KPair *kp;
    const double *eps;
    hipGraphExec_t exec;
    struct Stamp {
      int step, id, slot;  // iteration in the chunk, kernel, stamp pair
    };
    std::vector<Stamp> stamps;
  };
  std::vector<CgGraph> graphs;
  bool capturing = false;
  int capture_step = 0;
  std::vector<CgGraph::Stamp> capture_stamps;
  // Timing inside graphs: events recorded by graph nodes cannot be queried, so a one-thread
  // kernel writes the constant-rate device clock before and after each timed kernel.
  unsigned long long *d_stamps = nullptr;
  double clock_khz = 0.0;
  // Launch shapes chosen by timing candidates on this device (tune_* below): per GEMM
  // shape (precision, rows, batch) the projection tile, its K split and the expansion band
  // tile; per precision the plane-batch variant of the local-potential FFT round trip.
  struct GemmChoice {
    int prec, M, nk;
    int tile, ns, bv;
    float proj_ms, expand_ms, proj_default_ms, expand_default_ms;
  };
  std::vector<GemmChoice> gemm_tuned;
  int plane_var[2] = {0, 0};  // [0] FP64, [1] FP32
  int stick_var[2][2] = {{0, 0}, {0, 0}};  // [precision][inverse, forward] z-transform variant
  float stick_ms[2][2][3] = {};
  bool stick_tuned[2] = {false, false};
  int plane_nvar[2] = {0, 0};
  float plane_ms[2][kPlaneVariants] = {};
  bool plane_tuned[2] = {false, false};
  int use_tuned = 0;  // hp_scf_params.autotune of the current call
  double *d_tol = nullptr;  // [0] tolerance of the FP64 CG, [1] of the FP32 inner CG
  int graph_chunk = 0;      // 0: kernels are launched one by one
  int prev_iters[2] = {0, 0};

  template <class T>
  hp_status alloc(T **p, size_t count) {
    HPTRY(dalloc(p, count));
    allocs.push_back((void *)*p);
    return HP_OK;
  }
};

namespace {

constexpr int kNmixMax = 8;
// Sternheimer tolerance of SCF iteration i > 1: kAdaptiveTol x (mixing residual of i-1).
constexpr double kAdaptiveTol = 1e-2;
// Mixed precision: outer tolerances at or above this are met by the FP32 inner solve alone.
// Default of hp_scf_params.lowp_trust_tol.
constexpr double kFp32TrustTol = 1e-6;

enum KernelId {
  K_STICK_INV = 0,
  K_PLANE_VLOC,
  K_STICK_FWD,
  K_ZPROJ,
  K_ZEXPAND,
  K_CG_STEP,
  K_PLANE_DRHO,
  K_PLANE_MUL,
  K_STICK_INV32,
  K_PLANE_VLOC32,
  K_STICK_FWD32,
  K_ZPROJ32,
  K_ZEXPAND32,
  K_CG_STEP32,
  K_ZPROJ_REDUCE,
  K_CG_INIT,
  K_RESIDUAL64,
  K_REFINE,
  K_RHS,
  K_DRHO_STICKS,
  K_DRHO_REDUCE,
  K_HXC,
  K_DN,
  K_MIX,
  K_ZPROJ16,
  K_ZEXPAND16,
  K_PLANE_MUL32,
  K_PLANE_DRHO32,
  K_COUNT
};
static_assert(K_COUNT <= 32, "profile slots");
const char *const kKernelNames[K_COUNT] = {
    "stick_inv",   "plane_vloc",   "stick_fwd",   "zproj",       "zexpand",     "cg_step",
    "plane_drho",  "plane_mul_fwd", "stick_inv32", "plane_vloc32", "stick_fwd32", "zproj32",
    "zexpand32",   "cg_step32",    "zproj_reduce", "cg_init",     "residual64",  "refine_update",
    "rhs_other",   "drho_sticks",  "drho_reduce", "hxc",         "dn",          "mixing",
    "zproj16",     "zexpand16",    "plane_mul_fwd32", "plane_drho32"};

hipEvent_t prof_event(hp_ctx *c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

constexpr int kMaxStamps = 256;  // stamp pairs per captured chunk

// Enqueue `launch` bracketed by events (eager) or device-clock stamps (under graph
// capture) when profiling is on.
template <class F>
hipError_t timed(hp_ctx *c, int id, F launch) {
  if (!c->prof_on) return launch();
  if (c->capturing) {
    const int slot = (int)c->capture_stamps.size();
    if (slot >= kMaxStamps) return launch();
    hipError_t e = launch_clock_stamp(c->d_stamps + 2 * slot, c->stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = launch_clock_stamp(c->d_stamps + 2 * slot + 1, c->stream);
    if (e != hipSuccess) return e;
    c->capture_stamps.push_back({c->capture_step, id, slot});
    return hipSuccess;
  }
  hipEvent_t a = prof_event(c), b = prof_event(c);
  if (!a || !b) return launch();
  hipError_t e = hipEventRecord(a, c->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, c->stream);
  if (e != hipSuccess) return e;
  c->pending.push_back({id, a, b});
  return hipSuccess;
}

void prof_harvest(hp_ctx *c) {
  for (auto &p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof_calls[p.id] += 1;
      c->prof_ms[p.id] += ms;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

hp_status check_kpoint(const hp_kpoint &k, int i, const hp_ground_state *gs) {
  if (k.struct_size != sizeof(hp_kpoint)) return fail(HP_ERR_ARG, "kpts[%d].struct_size mismatch", i);
  if (k.npw < 1) return fail(HP_ERR_ARG, "kpts[%d].npw = %d", i, k.npw);
  if (!k.miller || !k.eps || !k.u || !k.beta) return fail(HP_ERR_ARG, "kpts[%d] has a NULL array", i);
  if (gs->projectors == HP_PROJ_ATOMIC && !k.phi) return fail(HP_ERR_ARG, "kpts[%d].phi is NULL", i);
  if (gs->projectors == HP_PROJ_ORTHO_ATOMIC && !k.atwfc) return fail(HP_ERR_ARG, "kpts[%d].atwfc is NULL", i);
  if (!(k.weight >= 0.0)) return fail(HP_ERR_ARG, "kpts[%d].weight < 0", i);
  return HP_OK;
}

// Eigen-decomposition of a real symmetric n x n matrix by cyclic Jacobi rotations: on
// return a is diagonal (the eigenvalues) and the columns of v are the eigenvectors.
bool jacobi_eigen(int n, std::vector<double> &a, std::vector<double> &v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? diag : off) += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    if (off <= 1e-30 * diag) return true;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (apq == 0.0) continue;
        // rotation in the (p, q) plane that zeroes a_pq: t = tan of the angle, the smaller
        // root of t^2 + 2 theta t - 1 = 0
        const double theta = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = cs * akp - sn * akq;
          a[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = cs * apk - sn * aqk;
          a[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = cs * vkp - sn * vkq;
          v[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  return false;
}

// Cold (Marzari-Vanderbilt) smearing of x = (e_F - e) / sigma: occupation, its derivative,
// and the smooth step (1 + erf(x)) / 2 that splits pairs of states.
double cold_occ(double x) {
  const double u = x - 1.0 / std::sqrt(2.0);
  return 0.5 * (1.0 + std::erf(u)) + std::exp(-u * u) / std::sqrt(2.0 * M_PI);
}
double cold_delta(double x) {
  const double u = x - 1.0 / std::sqrt(2.0);
  return std::exp(-u * u) * (1.0 - std::sqrt(2.0) * u) / std::sqrt(M_PI);
}
double split_step(double x) { return 0.5 * (1.0 + std::erf(x)); }

// Eigenpairs of a Hermitian n x n matrix (row-major complex): lam ascending, column a of V
// (V[m * n + a]) the eigenvector of lam[a].  Through the real symmetric embedding, whose
// spectrum is that of M with every eigenvalue twice; the embedding eigenvectors [x; y] are
// read as complex vectors x + i y and made orthonormal over the complex numbers in
// ascending eigenvalue order, keeping the n that are independent.
bool herm_eig(int n, const std::complex<double> *M, double *lam, std::complex<double> *V) {
  const int m = 2 * n;
  std::vector<double> a((size_t)m * m), w;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const std::complex<double> z = M[(size_t)i * n + j];
      a[(size_t)i * m + j] = a[(size_t)(i + n) * m + j + n] = z.real();
      a[(size_t)i * m + j + n] = -z.imag();
      a[(size_t)(i + n) * m + j] = z.imag();
    }
  if (!jacobi_eigen(m, a, w)) return false;
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return a[(size_t)x * m + x] < a[(size_t)y * m + y]; });
  int got = 0;
  std::vector<std::complex<double>> v(n);
  for (int t = 0; t < m && got < n; ++t) {
    const int k = order[t];
    for (int i = 0; i < n; ++i) v[i] = {w[(size_t)i * m + k], w[(size_t)(i + n) * m + k]};
    for (int b = 0; b < got; ++b) {  // remove the components along accepted vectors
      std::complex<double> d = 0.0;
      for (int i = 0; i < n; ++i) d += std::conj(V[(size_t)i * n + b]) * v[i];
      for (int i = 0; i < n; ++i) v[i] -= d * V[(size_t)i * n + b];
    }
    double nn = 0.0;
    for (int i = 0; i < n; ++i) nn += std::norm(v[i]);
    if (nn < 0.25) continue;  // dependent over the complex numbers on an accepted vector
    nn = std::sqrt(nn);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + got] = v[i] / nn;
    lam[got++] = a[(size_t)k * m + k];
  }
  return got == n;
}

// X = O^-1/2 of a Hermitian positive-definite n x n matrix (row-major complex), through
// its real symmetric embedding [[Re O, -Im O], [Im O, Re O]], on which functions act
// as on O.  Returns false if O is not positive definite to working precision.
bool inv_sqrt_hermitian(int n, const std::complex<double> *O, std::complex<double> *X) {
  const int m = 2 * n;
  std::vector<double> a((size_t)m * m), v;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const std::complex<double> z = O[(size_t)i * n + j];
      a[(size_t)i * m + j] = z.real();
      a[(size_t)(i + n) * m + j + n] = z.real();
      a[(size_t)i * m + j + n] = -z.imag();
      a[(size_t)(i + n) * m + j] = z.imag();
    }
  if (!jacobi_eigen(m, a, v)) return false;
  double lmax = 0.0, lmin = 1e300;
  for (int i = 0; i < m; ++i) {
    lmax = std::max(lmax, a[(size_t)i * m + i]);
    lmin = std::min(lmin, a[(size_t)i * m + i]);
  }
  if (!(lmin > 1e-12 * lmax)) return false;
  std::vector<double> f(m);
  for (int i = 0; i < m; ++i) f[i] = 1.0 / std::sqrt(a[(size_t)i * m + i]);
  for (int i = 0; i < n; ++i)  // F = V f(L) V^T; X = F[:n,:n] + i F[n:,:n]
    for (int j = 0; j < n; ++j) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < m; ++k) {
        re += v[(size_t)i * m + k] * f[k] * v[(size_t)j * m + k];
        im += v[(size_t)(i + n) * m + k] * f[k] * v[(size_t)j * m + k];
      }
      X[(size_t)i * n + j] = {re, im};
    }
  return true;
}

// Host-side view of one k-entry after sorting plane waves into z-sticks.
struct Layout {
  std::vector<int> order;         // internal -> caller
  std::vector<int> sx, sy, sstart, slen, iz, xa;
  int mext[2] = {0, 0};           // x, y: max(m + 1, -m) over the plane waves
};

hp_status build_layout(const hp_kpoint &k, int n1, int n2, int n3, Layout &L, int idx) {
  const int npw = k.npw;
  std::vector<long> key(npw);
  int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  for (int p = 0; p < npw; ++p) {
    for (int d = 0; d < 3; ++d) {
      mn[d] = std::min(mn[d], k.miller[3 * p + d]);
      mx[d] = std::max(mx[d], k.miller[3 * p + d]);
    }
  }
  const int N[3] = {n1, n2, n3};
  for (int d = 0; d < 2; ++d) L.mext[d] = npw > 0 ? std::max(mx[d] + 1, -mn[d]) : 0;
  for (int d = 0; d < 3; ++d)
    if (mx[d] - mn[d] + 1 > N[d])
      return fail(HP_ERR_SHAPE, "kpts[%d]: sphere spans %d along axis %d, grid has %d", idx, mx[d] - mn[d] + 1, d, N[d]);
  for (int p = 0; p < npw; ++p) {
    const int x = wrapi(k.miller[3 * p], n1), y = wrapi(k.miller[3 * p + 1], n2), z = wrapi(k.miller[3 * p + 2], n3);
    key[p] = ((long)x * n2 + y) * n3 + z;
  }
  L.order.resize(npw);
  std::iota(L.order.begin(), L.order.end(), 0);
  std::sort(L.order.begin(), L.order.end(), [&](int a, int b) { return key[a] < key[b]; });
  for (int p = 1; p < npw; ++p)
    if (key[L.order[p]] == key[L.order[p - 1]]) return fail(HP_ERR_SHAPE, "kpts[%d]: repeated plane wave", idx);
  long last_col = -1;
  for (int p = 0; p < npw; ++p) {
    const long kk = key[L.order[p]];
    const long col = kk / n3;
    if (col != last_col) {
      L.sx.push_back((int)(col / n2));
      L.sy.push_back((int)(col % n2));
      L.sstart.push_back(p);
      L.slen.push_back(0);
      if (L.xa.empty() || L.xa.back() != (int)(col / n2)) L.xa.push_back((int)(col / n2));
      last_col = col;
    }
    L.slen.back()++;
    L.iz.push_back((int)(kk % n3));
  }
  return HP_OK;
}

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double s() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

hp_status sync(hp_ctx *c) {
  HPCHK(hipStreamSynchronize(c->stream));
  if (!c->pending.empty()) prof_harvest(c);
  return HP_OK;
}

// nsplit for the projection GEMM so that a launch has enough workgroups.
int choose_nsplit(int M, int nb, int nk, int npw_max) {
  const int tiles = ((M + 31) / 32) * ((nb + 31) / 32) * nk;
  int ns = (2048 + tiles - 1) / tiles;
  ns = std::max(1, std::min(ns, 16));
  while (ns > 1 && npw_max / ns < 256) --ns;
  return ns;
}

// Launch shape of a GEMM: the tuned one when tuning is on and the shape has been tuned,
// else 32x32 projection tiles, the K split of choose_nsplit and 32-band expansion tiles.
struct GemmShape {
  int tile, ns, bv;
};
GemmShape gemm_shape(const hp_ctx *c, int prec, int M, int nk) {
  if (c->use_tuned)
    for (const auto &g : c->gemm_tuned)
      if (g.prec == prec && g.M == M && g.nk == nk) return {g.tile, g.ns, g.bv};
  return {0, choose_nsplit(M, c->n_occ, nk, c->npw_max), 1};
}
int plane_variant(const hp_ctx *c, int prec) { return c->use_tuned ? c->plane_var[prec == 32 ? 1 : 0] : 0; }
int stick_variant(const hp_ctx *c, int prec, int fwd) { return c->use_tuned ? c->stick_var[prec == 32][fwd] : 0; }

// C[k][m][v] = scale_m * sum_G conj(T[m0+m][G]) X[k,v][G]  (K-split partials in cpart, or the
// context's buffer)
hp_status proj(hp_ctx *c, const KPair *kp, int use_kq, int nk, const double2 *T, long tstride, int m0, int M,
               const double2 *X, int nb, const double *row_scale, double gscale, double2 *Cout,
               const int *active = nullptr, double2 *cpart = nullptr) {
  const GemmShape gs = gemm_shape(c, 64, M, nk);
  const int ns = gs.ns;
  double2 *cp = cpart ? cpart : c->Cpart;
  HPCHK(timed(c, K_ZPROJ, [&] {
    return launch_zproj(kp, use_kq, nk, T, tstride, m0, M, X, c->ld, nb, c->d_npw, cp, ns, active, gs.tile,
                        c->stream);
  }));
  HPCHK(timed(c, K_ZPROJ_REDUCE, [&] {
    return launch_zproj_reduce(nk, M, nb, ns, cp, row_scale, gscale, Cout, c->stream);
  }));
  return HP_OK;
}

// Intermediate buffers of one operator apply: z-stick data before and after the plane
// round trip, projection partial sums (K split) and projections.
struct OpWork {
  double2 *S1, *S2, *Cpart, *C;
};

// Y = (H_{k+q} + alpha P_v - eps_v) X over nitems (or H_k X for diagnostics when eps == nullptr,
// rows = n_beta only).  w: intermediate buffers (null: the context's).
hp_status apply_op(hp_ctx *c, const KPair *kp, int use_kq, int nk, int nb, const double2 *Xin, double2 *Y,
                   const double *eps, int rows, const int *active = nullptr, const OpWork *w = nullptr) {
  const int nitems = nk * nb;
  const OpWork wk = w ? *w : OpWork{c->S1, c->S2, c->Cpart, c->C};
  // the GEMM tiles cover the active bands only, packed per k
  const int *gmap = nullptr;
  if (active) {
    HPCHK(launch_active_map(active, nk, nb, c->bmap, c->stream));
    gmap = c->bmap;
  }
  HPCHK(timed(c, K_STICK_INV, [&] {
    return launch_stick_inv(c->sk, kp, use_kq, nb, nitems, Xin, c->ld, wk.S1, c->ns_pad, c->n3, c->az.tw,
                            c->max_chunk_pw, c->ns_max, active, stick_variant(c, 64, 0), c->stream);
  }));
  HPCHK(timed(c, K_PLANE_VLOC, [&] {
    return launch_plane_vloc(c->pl, c->sk, kp, use_kq, nb, nitems, wk.S1, wk.S2, c->ns_pad, c->d_vp, active,
                             plane_variant(c, 64), c->stream);
  }));
  HPCHK(timed(c, K_STICK_FWD, [&] {
    return launch_stick_fwd(c->sk, kp, use_kq, nb, nitems, wk.S2, c->ns_pad, c->n3, c->az.tw, 1.0 / (double)c->nr,
                            Y, c->ld, 0, c->d_kin, eps, Xin, nb, c->max_chunk_pw, c->ns_max, active,
                            stick_variant(c, 64, 1), c->stream);
  }));
  HPTRY(proj(c, kp, use_kq, nk, c->d_T, c->t_stride, 0, rows, Xin, nb, c->d_rowscale, 1.0, wk.C, gmap, wk.Cpart));
  HPCHK(timed(c, K_ZEXPAND, [&] {
    return launch_zexpand(kp, use_kq, nk, c->d_T, c->t_stride, 0, rows, wk.C, (long)rows * nb, 1.0, Y, c->ld, nb,
                          c->d_npw, c->npw_max, gmap, gemm_shape(c, 64, rows, nk).bv, c->stream);
  }));
  return HP_OK;
}

// RHS of Eq. 15 for nk pairs: B = -P_c (dv psi + V_pert psi); dv may be null.  lowp: the
// product dv psi and its transform in FP32 (psi from the FP32 copy), the rest in FP64.
hp_status build_rhs(hp_ctx *c, const KPair *kp, int nk, int site, const double2 *dv, const double2 *psi,
                    bool lowp = false) {
  const int nb = c->n_occ, nitems = nk * nb;
  if (dv && lowp) {
    float2 *S1 = reinterpret_cast<float2 *>(c->S1);
    HPCHK(launch_to_f32((const double *)dv, (float *)c->dv32, 2L * c->nspin * c->nr, c->stream));
    HPCHK(timed(c, K_PLANE_MUL32, [&] {
      return launch_plane_mul_fwd32(c->pl32, c->sk, kp, nb, nitems, c->psi32, c->dv32, S1, c->ns_pad, c->stream);
    }));
    HPCHK(timed(c, K_RHS, [&] {
      return launch_stick_fwd32(c->sk, kp, 1, nb, nitems, S1, c->ns_pad, c->n3, c->az32.tw32, -1.0 / (double)c->nr,
                                c->AP32, c->ld, 2, nullptr, nullptr, nullptr, nb, c->max_chunk_pw, c->ns_max, nullptr,
                                stick_variant(c, 32, 1), c->stream);
    }));
    HPCHK(launch_to_f64((const float *)c->AP32, (double *)c->B, 2L * nitems * c->ld, c->stream));
  } else if (dv) {
    HPCHK(timed(c, K_PLANE_MUL, [&] {
      return launch_plane_mul_fwd(c->pl, c->sk, kp, nb, nitems, psi, dv, c->S1, c->ns_pad, c->stream);
    }));
    HPCHK(timed(c, K_RHS, [&] {
      return launch_stick_fwd(c->sk, kp, 1, nb, nitems, c->S1, c->ns_pad, c->n3, c->az.tw, -1.0 / (double)c->nr, c->B,
                              c->ld, 2, nullptr, nullptr, nullptr, nb, c->max_chunk_pw, c->ns_max, nullptr,
                              stick_variant(c, 64, 1), c->stream);
    }));
  } else {
    HPCHK(hipMemsetAsync(c->B, 0, sizeof(double2) * (size_t)nitems * c->ld, c->stream));
  }
  // - sum_m |phi_{m,k+q}> <phi_{m,k}|u_vk>   (Eq. 16)
  HPCHK(timed(c, K_RHS, [&] {
    return launch_zexpand(kp, 1, nk, c->d_phi, c->phi_stride, 5 * site, 5, c->d_A + (size_t)5 * site * nb,
                          (long)5 * c->n_hub * nb, -1.0, c->B, c->ld, nb, c->d_npw, c->npw_max, nullptr,
                          gemm_shape(c, 64, 5, nk).bv, c->stream);
  }));
  // P_c = 1 - sum_v' |u_v',k+q><u_v',k+q|   (Eq. 18)
  HPTRY(proj(c, kp, 1, nk, c->d_T, c->t_stride, c->n_beta, c->n_occ, c->B, nb, nullptr, 1.0, c->C));
  if (c->degauss > 0.0) {
    // metals: B_i = f_i B_i - sum_j beta_ij u_j <u_j|B_i> (B = -(dV + V_pert) u)
    if (c->metal_q0) {  // Fermi-level shift from <u_i|dV|u_i> = -C[k][i][i]
      std::vector<double2> h((size_t)nk * nb * nb);
      HPCHK(hipMemcpyAsync(h.data(), c->C, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, c->stream));
      HPTRY(sync(c));
      std::complex<double> num = 0.0;
      double den = 0.0;
      for (int k = 0; k < nk; ++k)
        for (int i = 0; i < nb; ++i) {
          const double w = c->ent[k].weight * c->occ_d[(size_t)k * nb + i];
          const double2 d = h[((size_t)k * nb + i) * nb + i];
          num -= w * std::complex<double>(d.x, d.y);
          den += w;
        }
      c->fermi_shift = den != 0.0 ? num / den : std::complex<double>(0.0);
    }
    HPCHK(launch_scale_rows((long)nk * nb * nb, 1, c->d_beta, c->C, c->stream));
    HPCHK(launch_scale_rows((long)nitems * c->ld, c->ld, c->d_focc, c->B, c->stream));
  }
  HPCHK(timed(c, K_RHS, [&] {
    return launch_zexpand(kp, 1, nk, c->d_T, c->t_stride, c->n_beta, c->n_occ, c->C, (long)c->n_occ * nb, -1.0, c->B,
                          c->ld, c->n_occ, c->d_npw, c->npw_max, nullptr, gemm_shape(c, 64, c->n_occ, nk).bv,
                          c->stream);
  }));
  return HP_OK;
}

hp_status apply_op32(hp_ctx *c, const KPair *kp, int nk, int nb, const float2 *Xin, float2 *Y, const double *eps,
                     int rows, const int *active);

constexpr int kMaxChunk = 8;  // CG iterations per captured graph at most

// Counter slots in c->count: [1] items with a non-finite residual (whole chunk),
// [2] / [3] items above tolerance / non-finite after the mixed-precision FP64 residual,
// [4 + i] items still above tolerance after iteration i of the chunk.
constexpr int kCntBad = 1, kCntResid = 2, kCntStep = 4;

// Enqueue `len` CG iterations of one precision (kind 0: FP64 operator and vectors,
// kind 1: FP32 inner solve) on c->stream. Items that have converged are skipped by every
// kernel, so iterations past convergence change nothing.
hp_status cg_enqueue_chunk(hp_ctx *c, int kind, int len, const KPair *kp, int nk, const double *eps_items) {
  const int nb = c->n_occ, nitems = nk * nb, rows = c->n_beta + c->n_occ;
  HPCHK(launch_fill_int(c->count, kCntStep + len, 0, c->stream));
  for (int i = 0; i < len; ++i) {
    c->capture_step = i;
    if (kind == 0) {
      HPTRY(apply_op(c, kp, 1, nk, nb, c->P, c->AP, eps_items, rows, c->active));
      HPCHK(timed(c, K_CG_STEP, [&] {
        return launch_cg_step(kp, nb, nitems, c->X, c->R, c->P, c->AP, c->d_diag, eps_items, c->ld, c->d_npw, c->ld,
                              c->rz, c->bn, c->rn, c->active, c->d_tol, c->count + kCntStep + i, c->count + kCntBad,
                              c->stream);
      }));
    } else {
      HPTRY(apply_op32(c, kp, nk, nb, c->P32, c->AP32, eps_items, rows, c->act_in));
      HPCHK(timed(c, K_CG_STEP32, [&] {
        return launch_cg_step32(kp, nb, nitems, c->X32, c->R32, c->P32, c->AP32, c->d_diag, eps_items, c->ld,
                                c->d_npw, c->ld, c->rz_in, c->bn_in, c->rn_in, c->act_in, c->d_tol + 1,
                                c->count + kCntStep + i, c->count + kCntBad, c->floor_in, c->stream);
      }));
    }
  }
  c->capture_step = 0;
  return HP_OK;
}

// The executable graph of a chunk, captured on first use.
hp_status cg_graph(hp_ctx *c, int kind, int len, const KPair *kp, int nk, const double *eps_items,
                   hp_ctx::CgGraph **out) {
  const int prof = c->prof_on ? 1 : 0;
  for (auto &g : c->graphs)
    if (g.kind == kind && g.len == len && g.prof == prof && g.nk == nk && g.lowp == c->lowp_gemm &&
        g.tuned == c->use_tuned && g.kp == kp && g.eps == eps_items) {
      *out = &g;
      return HP_OK;
    }
  if (c->graphs.size() >= 24) {  // bounded cache: drop the oldest
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  HPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  c->capture_stamps.clear();
  const hp_status st = cg_enqueue_chunk(c, kind, len, kp, nk, eps_items);
  c->capturing = false;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &graph);
  if (st != HP_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    c->capture_stamps.clear();
    if (st != HP_OK) return st;
    HPCHK(e);
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HPCHK(ei);
  c->graphs.push_back(
      {kind, len, prof, nk, c->lowp_gemm, c->use_tuned, kp, eps_items, exec, std::move(c->capture_stamps)});
  c->capture_stamps.clear();
  *out = &c->graphs.back();
  return HP_OK;
}

// Run one chunk of up to `len` iterations, eagerly or from its graph. On return: *steps =
// iterations that had work (the eager loop would have run exactly these), *stepped = items
// those iterations processed, *left = items still above tolerance.
hp_status cg_run_chunk(hp_ctx *c, int kind, int len, const KPair *kp, int nk, const double *eps_items, int active0,
                       int *steps, long *stepped, int *left) {
  hp_ctx::CgGraph *g = nullptr;
  if (c->graph_chunk > 0) {
    HPTRY(cg_graph(c, kind, len, kp, nk, eps_items, &g));
    HPCHK(hipGraphLaunch(g->exec, c->stream));
  } else {
    HPTRY(cg_enqueue_chunk(c, kind, len, kp, nk, eps_items));
  }
  int h[kCntStep + kMaxChunk];
  HPCHK(hipMemcpyAsync(h, c->count, sizeof(int) * (kCntStep + len), hipMemcpyDeviceToHost, c->stream));
  std::vector<unsigned long long> stamps;
  if (g && g->prof && !g->stamps.empty()) {
    stamps.resize(2 * g->stamps.size());
    HPCHK(hipMemcpyAsync(stamps.data(), c->d_stamps, sizeof(unsigned long long) * stamps.size(),
                         hipMemcpyDeviceToHost, c->stream));
  }
  HPTRY(sync(c));
  if (h[kCntBad] > 0) return fail(HP_ERR_NUMERIC, "non-finite residual in the Sternheimer solve");
  int n = 0, entry = active0;
  long done = 0;
  for (int i = 0; i < len && entry > 0; ++i) {
    ++n;
    done += entry;
    entry = h[kCntStep + i];
  }
  if (!stamps.empty()) {  // per-kernel times of the iterations that had work
    for (const auto &t : g->stamps) {
      if (t.step >= n) continue;
      const unsigned long long a = stamps[2 * t.slot], b = stamps[2 * t.slot + 1];
      c->prof_calls[t.id] += 1;
      c->prof_ms[t.id] += b > a ? (double)(b - a) / c->clock_khz : 0.0;
    }
  }
  *steps = n;
  *stepped = done;
  *left = entry;
  return HP_OK;
}

// Iterations for the next chunk: a power of two no larger than graph_chunk, the iterations
// left to max_it, or what the previous solve of this kind suggests is still to come.
int chunk_len(hp_ctx *c, int kind, int it, int max_it) {
  if (c->graph_chunk <= 0) return 1;
  int want = c->prev_iters[kind] > 0 ? c->prev_iters[kind] - it : c->graph_chunk;
  want = std::max(1, std::min(want, std::min(max_it - it, c->graph_chunk)));
  int len = 1;
  while (len * 2 <= want) len *= 2;
  return len;
}

hp_status set_tol(hp_ctx *c, int slot, double tol) {
  HPCHK(launch_fill_double(c->d_tol + slot, 1, tol, c->stream));
  return HP_OK;
}

// Batched preconditioned CG on (H_{k+q} + alpha O_{k+q} - eps_vk) X = B (Eq. 15).
hp_status cg_solve(hp_ctx *c, const KPair *kp, int nk, const double *eps_items, int warm, double tol, int max_it,
                   int *iters, int *not_conv, double *max_rel, long *happ) {
  const int nb = c->n_occ, nitems = nk * nb;
  const int rows = c->n_beta + c->n_occ;
  c->ax_valid = false;  // X changes below
  if (warm) HPTRY(apply_op(c, kp, 1, nk, nb, c->X, c->AP, eps_items, rows));
  if (warm) *happ += nitems;
  HPCHK(timed(c, K_CG_INIT, [&] {
    return launch_cg_init(kp, nb, nitems, c->B, c->X, c->R, c->P, c->AP, warm, c->d_diag, eps_items, c->ld, c->d_npw,
                          c->ld, c->rz, c->bn, c->rn, c->active, tol, c->stream);
  }));
  HPTRY(set_tol(c, 0, tol));
  int it = 0, left = 0;
  {
    std::vector<int> act(nitems);
    HPCHK(hipMemcpyAsync(act.data(), c->active, sizeof(int) * nitems, hipMemcpyDeviceToHost, c->stream));
    HPTRY(sync(c));
    for (int a : act) left += a;
  }
  while (left > 0 && it < max_it) {
    int steps = 0;
    long stepped = 0;
    HPTRY(cg_run_chunk(c, 0, chunk_len(c, 0, it, max_it), kp, nk, eps_items, left, &steps, &stepped, &left));
    it += steps;
    *happ += stepped;  // converged items are skipped by the operator kernels
  }
  c->prev_iters[0] = it;
  *iters = it;
  *not_conv = left;
  std::vector<double> rn(nitems), bn(nitems);
  HPCHK(hipMemcpyAsync(rn.data(), c->rn, sizeof(double) * nitems, hipMemcpyDeviceToHost, c->stream));
  HPCHK(hipMemcpyAsync(bn.data(), c->bn, sizeof(double) * nitems, hipMemcpyDeviceToHost, c->stream));
  HPTRY(sync(c));
  double m = 0.0;
  for (int i = 0; i < nitems; ++i)
    if (bn[i] > 0) m = std::max(m, rn[i] / bn[i]);
  *max_rel = m;
  return HP_OK;
}

// FP32 tables and buffers for the mixed-precision inner solves (once per context).
hp_status setup32(hp_ctx *c) {
  if (c->have32) return HP_OK;
  const long nitems = (long)c->n_mesh * c->n_occ;
  const size_t vec = (size_t)nitems * c->ld;
  const long ntw = c->n1 + c->n2 + c->n3;
  HPTRY(c->alloc(&c->tw32, ntw));
  HPCHK(launch_to_f32((const double *)c->tw, (float *)c->tw32, 2 * ntw, c->stream));
  HPTRY(c->alloc(&c->T32, (size_t)c->n_kpts * c->t_stride));
  HPCHK(launch_to_f32((const double *)c->d_T, (float *)c->T32, 2L * c->n_kpts * c->t_stride, c->stream));
  HPTRY(c->alloc(&c->vp32, (size_t)c->nspin * c->nr));
  HPCHK(launch_to_f32(c->d_vp, c->vp32, (long)c->nspin * c->nr, c->stream));
  for (float2 **b : {&c->X32, &c->R32, &c->B32, &c->P32, &c->AP32}) {
    HPTRY(c->alloc(b, vec));
    HPCHK(hipMemsetAsync(*b, 0, sizeof(float2) * vec, c->stream));
  }
  HPTRY(c->alloc(&c->AX, vec));
  c->ax_valid = false;
  HPTRY(c->alloc(&c->bn_in, nitems));
  HPTRY(c->alloc(&c->rn_in, nitems));
  HPTRY(c->alloc(&c->rz_in, nitems));
  HPTRY(c->alloc(&c->floor_in, nitems));
  HPTRY(c->alloc(&c->act_in, nitems));
  HPTRY(c->alloc(&c->act_out, nitems));
  // FP32 copy of the occupied states on the grid and a response-potential buffer: the
  // RHS product and the response density of iterations solved to >= 1e-6 run in FP32
  HPTRY(c->alloc(&c->psi32, (size_t)c->n_mesh * c->n_occ * c->nr));
  HPCHK(launch_to_f32((const double *)c->d_psi, (float *)c->psi32, 2L * c->n_mesh * c->n_occ * c->nr, c->stream));
  HPTRY(c->alloc(&c->dv32, (size_t)c->nspin * c->nr));
  c->pl32 = c->pl;
  c->pl32.ax.tw32 = c->tw32;
  c->pl32.ay.tw32 = c->tw32 + c->n1;
  c->az32 = c->az;
  c->az32.tw32 = c->tw32 + c->n1 + c->n2;
  HPTRY(sync(c));
  c->have32 = true;
  return HP_OK;
}

// Packed-bfloat16 copy of the stacked projector table (once per context).
hp_status setup16(hp_ctx *c) {
  if (c->T16) return HP_OK;
  unsigned *t = nullptr;
  HPTRY(c->alloc(&t, (size_t)c->n_kpts * c->t_stride));
  HPCHK(launch_to_bf16_pairs(c->d_T, t, (long)c->n_kpts * c->t_stride, c->stream));
  HPTRY(sync(c));
  c->T16 = t;
  return HP_OK;
}

// Y = (H_{k+q} + alpha P_v - eps_v) X in FP32 (FP32 FFTs; FP32 or BF16 MFMA GEMMs with FP32 accumulation).
hp_status apply_op32(hp_ctx *c, const KPair *kp, int nk, int nb, const float2 *Xin, float2 *Y, const double *eps,
                     int rows, const int *active) {
  const int nitems = nk * nb;
  const int *gmap = nullptr;  // the GEMM tiles cover the active bands only, packed per k
  if (active) {
    HPCHK(launch_active_map(active, nk, nb, c->bmap, c->stream));
    gmap = c->bmap;
  }
  float2 *S1 = reinterpret_cast<float2 *>(c->S1), *S2 = reinterpret_cast<float2 *>(c->S2);
  float2 *Cpart = reinterpret_cast<float2 *>(c->Cpart), *C = reinterpret_cast<float2 *>(c->C);
  HPCHK(timed(c, K_STICK_INV32, [&] {
    return launch_stick_inv32(c->sk, kp, 1, nb, nitems, Xin, c->ld, S1, c->ns_pad, c->n3, c->az32.tw32,
                              c->max_chunk_pw, c->ns_max, active, stick_variant(c, 32, 0), c->stream);
  }));
  HPCHK(timed(c, K_PLANE_VLOC32, [&] {
    return launch_plane_vloc32(c->pl32, c->sk, kp, 1, nb, nitems, S1, S2, c->ns_pad, c->vp32, active,
                               plane_variant(c, 32), c->stream);
  }));
  HPCHK(timed(c, K_STICK_FWD32, [&] {
    return launch_stick_fwd32(c->sk, kp, 1, nb, nitems, S2, c->ns_pad, c->n3, c->az32.tw32, 1.0 / (double)c->nr, Y,
                              c->ld, 0, c->d_kin, eps, Xin, nb, c->max_chunk_pw, c->ns_max, active,
                              stick_variant(c, 32, 1), c->stream);
  }));
  // rows [0, m16) of the stacked table in BF16, rows [m16, rows) in FP32
  const int m16 = c->lowp_gemm == HP_GEMM_BF16 ? rows : c->lowp_gemm == HP_GEMM_BF16_PV32 ? c->n_beta : 0;
  if (m16 > 0) {
    const GemmShape g16 = gemm_shape(c, 16, m16, nk);
    HPCHK(timed(c, K_ZPROJ16, [&] {
      return launch_zproj16(kp, 1, nk, c->T16, c->t_stride, 0, m16, Xin, c->ld, nb, c->d_npw, Cpart, g16.ns, gmap,
                            g16.tile, c->stream);
    }));
    HPCHK(timed(c, K_ZPROJ_REDUCE, [&] {
      return launch_zproj_reduce32(nk, m16, nb, g16.ns, Cpart, c->d_rowscale, 1.0, C, c->stream);
    }));
    HPCHK(timed(c, K_ZEXPAND16, [&] {
      return launch_zexpand16(kp, 1, nk, c->T16, c->t_stride, 0, m16, C, (long)m16 * nb, 1.0, Y, c->ld, nb,
                              c->d_npw, c->npw_max, gmap, g16.bv, c->stream);
    }));
  }
  if (m16 < rows) {
    const int M = rows - m16;
    const GemmShape gs = gemm_shape(c, 32, M, nk);
    HPCHK(timed(c, K_ZPROJ32, [&] {
      return launch_zproj32(kp, 1, nk, c->T32, c->t_stride, m16, M, Xin, c->ld, nb, c->d_npw, Cpart, gs.ns, gmap,
                            gs.tile, c->stream);
    }));
    HPCHK(timed(c, K_ZPROJ_REDUCE, [&] {
      return launch_zproj_reduce32(nk, M, nb, gs.ns, Cpart, c->d_rowscale + m16, 1.0, C, c->stream);
    }));
    HPCHK(timed(c, K_ZEXPAND32, [&] {
      return launch_zexpand32(kp, 1, nk, c->T32, c->t_stride, m16, M, C, (long)M * nb, 1.0, Y, c->ld, nb, c->d_npw,
                              c->npw_max, gmap, gs.bv, c->stream);
    }));
  }
  return HP_OK;
}

// ---------------------------------------------------------------- autotuner
// Candidates are timed on this device with the context's own buffers at the start of a
// call, before any of them holds state: the GEMMs write the K-split partials (Cpart), the
// projections (C) and the operator outputs (AP / AP32), the plane kernels the stick buffers
// (S1 / S2). The tile and plane-batch choices do not change any arithmetic; the K split
// changes the order of the partial sums (last-bit differences).

template <class F>
hp_status time_launch(hp_ctx *c, F launch, int reps, float *ms) {
  HPCHK(launch());  // warm-up (code load, caches)
  HPCHK(hipEventRecord(c->ev[10], c->stream));
  for (int r = 0; r < reps; ++r) HPCHK(launch());
  HPCHK(hipEventRecord(c->ev[11], c->stream));
  HPCHK(hipEventSynchronize(c->ev[11]));
  float t = 0.f;
  HPCHK(hipEventElapsedTime(&t, c->ev[10], c->ev[11]));
  *ms = t / (float)reps;
  return HP_OK;
}

hp_status tune_gemm(hp_ctx *c, int prec, int M, int nk) {
  for (const auto &g : c->gemm_tuned)
    if (g.prec == prec && g.M == M && g.nk == nk) return HP_OK;
  if (prec == 16) HPTRY(setup16(c));
  if (M > c->n_proj) return HP_OK;  // timed against the first M rows of the stacked table
  const int nb = c->n_occ;
  const KPair *kp = c->d_kp;
  const int ns_default = choose_nsplit(M, nb, nk, c->npw_max);
  hp_ctx::GemmChoice best{prec, M, nk, 0, ns_default, 1, 1e30f, 1e30f, 0.f, 0.f};
  std::vector<int> splits{ns_default};  // the default first, then powers of two
  for (int ns = 1; ns <= c->nsplit_cap && (ns == 1 || c->npw_max / ns >= 256); ns *= 2)
    if (ns != ns_default) splits.push_back(ns);
  for (int tile = 0; tile < 4; ++tile)
    for (int ns : splits) {
      float ms = 0.f;
      if (prec == 16 && tile != 0 && tile != 3) continue;  // BF16 tiles: 32x32 and 64x64
      if (prec == 64) {
        HPTRY(time_launch(c, [&] {
          hipError_t e = launch_zproj(kp, 1, nk, c->d_T, c->t_stride, 0, M, c->X, c->ld, nb, c->d_npw, c->Cpart, ns,
                                      nullptr, tile, c->stream);
          if (e != hipSuccess) return e;
          return launch_zproj_reduce(nk, M, nb, ns, c->Cpart, nullptr, 1.0, c->C, c->stream);
        }, 2, &ms));
      } else if (prec == 16) {
        float2 *Cpart = reinterpret_cast<float2 *>(c->Cpart), *C = reinterpret_cast<float2 *>(c->C);
        HPTRY(time_launch(c, [&] {
          hipError_t e = launch_zproj16(kp, 1, nk, c->T16, c->t_stride, 0, M, c->X32, c->ld, nb, c->d_npw, Cpart, ns,
                                        nullptr, tile, c->stream);
          if (e != hipSuccess) return e;
          return launch_zproj_reduce32(nk, M, nb, ns, Cpart, nullptr, 1.0, C, c->stream);
        }, 2, &ms));
      } else {
        float2 *Cpart = reinterpret_cast<float2 *>(c->Cpart), *C = reinterpret_cast<float2 *>(c->C);
        HPTRY(time_launch(c, [&] {
          hipError_t e = launch_zproj32(kp, 1, nk, c->T32, c->t_stride, 0, M, c->X32, c->ld, nb, c->d_npw, Cpart, ns,
                                        nullptr, tile, c->stream);
          if (e != hipSuccess) return e;
          return launch_zproj_reduce32(nk, M, nb, ns, Cpart, nullptr, 1.0, C, c->stream);
        }, 2, &ms));
      }
      if (tile == 0 && ns == ns_default) best.proj_default_ms = ms;
      if (ms < best.proj_ms) {
        best.proj_ms = ms;
        best.tile = tile;
        best.ns = ns;
      }
    }
  for (int bv = 1; bv <= 4; bv *= 2) {
    float ms = 0.f;
    if (prec == 64) {
      HPTRY(time_launch(c, [&] {
        return launch_zexpand(kp, 1, nk, c->d_T, c->t_stride, 0, M, c->C, (long)M * nb, 1.0, c->AP, c->ld, nb,
                              c->d_npw, c->npw_max, nullptr, bv, c->stream);
      }, 2, &ms));
    } else if (prec == 16) {
      const float2 *C = reinterpret_cast<const float2 *>(c->C);
      HPTRY(time_launch(c, [&] {
        return launch_zexpand16(kp, 1, nk, c->T16, c->t_stride, 0, M, C, (long)M * nb, 1.0, c->AP32, c->ld, nb,
                                c->d_npw, c->npw_max, nullptr, bv, c->stream);
      }, 2, &ms));
    } else {
      const float2 *C = reinterpret_cast<const float2 *>(c->C);
      HPTRY(time_launch(c, [&] {
        return launch_zexpand32(kp, 1, nk, c->T32, c->t_stride, 0, M, C, (long)M * nb, 1.0, c->AP32, c->ld, nb,
                                c->d_npw, c->npw_max, nullptr, bv, c->stream);
      }, 2, &ms));
    }
    if (bv == 1) best.expand_default_ms = ms;
    if (ms < best.expand_ms) {
      best.expand_ms = ms;
      best.bv = bv;
    }
  }
  c->gemm_tuned.push_back(best);
  return HP_OK;
}

hp_status tune_plane(hp_ctx *c, int prec, int nk) {
  const int slot = prec == 32 ? 1 : 0;
  if (c->plane_tuned[slot]) return HP_OK;
  const int nb = c->n_occ, nitems = nk * nb;
  const int csize = prec == 32 ? (int)sizeof(float2) : (int)sizeof(double2);
  const int nv = kPlaneVariants;
  float best = 1e30f;
  for (int v = 0; v < nv; ++v) {
    c->plane_ms[slot][v] = -1.f;  // not available for this grid
    if (!plane_vloc_variant_ok(c->pl, csize, v)) continue;
    float ms = 0.f;
    if (prec == 64) {
      HPTRY(time_launch(c, [&] {
        return launch_plane_vloc(c->pl, c->sk, c->d_kp, 1, nb, nitems, c->S1, c->S2, c->ns_pad, c->d_vp, nullptr, v,
                                 c->stream);
      }, 2, &ms));
    } else {
      float2 *S1 = reinterpret_cast<float2 *>(c->S1), *S2 = reinterpret_cast<float2 *>(c->S2);
      HPTRY(time_launch(c, [&] {
        return launch_plane_vloc32(c->pl32, c->sk, c->d_kp, 1, nb, nitems, S1, S2, c->ns_pad, c->vp32, nullptr, v,
                                   c->stream);
      }, 2, &ms));
    }
    c->plane_ms[slot][v] = ms;
    if (ms < best) {
      best = ms;
      c->plane_var[slot] = v;
    }
  }
  c->plane_nvar[slot] = nv;
  c->plane_tuned[slot] = true;
  return HP_OK;
}

// z transforms: a workgroup per 32 sticks, or a thread per stick (same sums, same order).
// z-transform variants available: the register ones need a compile-time N3 (24 or 40) and
// the staged one the plane waves of 256 sticks in LDS (at most 96 KB here, FP64 sizes).
int stick_variants(const hp_ctx *c) {
  if (c->n3 != 24 && c->n3 != 40) return 1;
  return (size_t)c->sk.max_pw256 * (sizeof(double2) + sizeof(int)) + c->n3 * sizeof(double2) <= 96 * 1024 ? 3 : 2;
}

hp_status tune_stick(hp_ctx *c, int prec, int nk) {
  const int slot = prec == 32 ? 1 : 0;
  if (c->stick_tuned[slot]) return HP_OK;
  const int nb = c->n_occ, nitems = nk * nb;
  const int nv = stick_variants(c);
  for (int fwd = 0; fwd < 2; ++fwd) {
    for (int v = nv; v < 3; ++v) c->stick_ms[slot][fwd][v] = -1.f;  // not available
    float best = 1e30f;
    for (int v = 0; v < nv; ++v) {
      float ms = 0.f;
      if (prec == 64) {
        HPTRY(time_launch(c, [&] {
          if (!fwd)
            return launch_stick_inv(c->sk, c->d_kp, 1, nb, nitems, c->X, c->ld, c->S1, c->ns_pad, c->n3, c->az.tw,
                                    c->max_chunk_pw, c->ns_max, nullptr, v, c->stream);
          return launch_stick_fwd(c->sk, c->d_kp, 1, nb, nitems, c->S2, c->ns_pad, c->n3, c->az.tw, 1.0, c->AP, c->ld,
                                  2, nullptr, nullptr, nullptr, nb, c->max_chunk_pw, c->ns_max, nullptr, v, c->stream);
        }, 2, &ms));
      } else {
        float2 *S1 = reinterpret_cast<float2 *>(c->S1), *S2 = reinterpret_cast<float2 *>(c->S2);
        HPTRY(time_launch(c, [&] {
          if (!fwd)
            return launch_stick_inv32(c->sk, c->d_kp, 1, nb, nitems, c->X32, c->ld, S1, c->ns_pad, c->n3,
                                      c->az32.tw32, c->max_chunk_pw, c->ns_max, nullptr, v, c->stream);
          return launch_stick_fwd32(c->sk, c->d_kp, 1, nb, nitems, S2, c->ns_pad, c->n3, c->az32.tw32, 1.0, c->AP32,
                                    c->ld, 2, nullptr, nullptr, nullptr, nb, c->max_chunk_pw, c->ns_max, nullptr, v,
                                    c->stream);
        }, 2, &ms));
      }
      c->stick_ms[slot][fwd][v] = ms;
      if (ms < best) {
        best = ms;
        c->stick_var[slot][fwd] = v;
      }
    }
  }
  c->stick_tuned[slot] = true;
  return HP_OK;
}

// Tune every launch shape a call on nk mesh points will use (c->d_kp must hold its pairs).
hp_status autotune(hp_ctx *c, int nk, int mixed) {
  if (!c->use_tuned) return HP_OK;
  const int rows = c->n_beta + c->n_occ;
  for (int M : {rows, c->n_occ, 5 * c->n_hub, 5}) HPTRY(tune_gemm(c, 64, M, nk));
  HPTRY(tune_plane(c, 64, nk));
  HPTRY(tune_stick(c, 64, nk));
  if (mixed) {
    HPTRY(setup32(c));
    if (c->lowp_gemm == HP_GEMM_FP32) HPTRY(tune_gemm(c, 32, rows, nk));
    if (c->lowp_gemm == HP_GEMM_BF16) HPTRY(tune_gemm(c, 16, rows, nk));
    if (c->lowp_gemm == HP_GEMM_BF16_PV32) {
      HPTRY(tune_gemm(c, 16, c->n_beta, nk));
      HPTRY(tune_gemm(c, 32, c->n_occ, nk));
    }
    HPTRY(tune_plane(c, 32, nk));
    HPTRY(tune_stick(c, 32, nk));
  }
  return HP_OK;
}

// Mixed precision: FP64 residual refinement around FP32 PCG inner solves.
//   r = B - A64 X ; while some ||r|| > tol ||B||: solve A32 d = r to inner_tol in FP32, X += d, recompute r.
hp_status cg_solve_mixed(hp_ctx *c, const KPair *kp, int nk, const double *eps_items, int warm, double tol,
                         int max_it, double inner_tol, int max_refine, double trust_tol, int *iters,
                         int *not_conv, double *max_rel, long *happ64, long *happ32, int *refines) {
  const int nb = c->n_occ, nitems = nk * nb;
  const int rows = c->n_beta + c->n_occ;
  HPTRY(setup32(c));
  if (c->lowp_gemm != HP_GEMM_FP32) HPTRY(setup16(c));
  int it_in = 0, nact = 0, ref = 0;
  bool trusted = false;
  int h_count[kCntStep] = {0};
  // At or above trust_tol (default 1e-6) the FP32 operator (FP32 GEMMs) is accurate to
  // ~1e-7 of |A X| ~ |B|, far below the tolerance: the warm-start residual then comes from
  // it, and the inner solve's own residual stands for the final one (no FP64 operator
  // apply at all).
  const bool trust = c->lowp_gemm == HP_GEMM_FP32 && tol >= trust_tol;
  // A warm start whose X is the last solve's final one, which ended on an FP64 residual:
  // A X is already in c->AX (the same operator, bit for bit the same product).
  const bool reuse_ax = warm && c->ax_valid;
  c->ax_valid = false;
  bool ax_fresh = false;  // c->AX = A X for the current X
  for (ref = 0; ref <= max_refine; ++ref) {
    const int have_x = warm || ref > 0;
    const bool reused = have_x && ref == 0 && reuse_ax;
    const bool ax32 = have_x && trust && ref == 0 && !reused;
    if (ax32) {
      HPCHK(launch_to_f32((const double *)c->X, (float *)c->X32, 2L * nitems * c->ld, c->stream));
      HPTRY(apply_op32(c, kp, nk, nb, c->X32, c->AP32, eps_items, rows, nullptr));
      *happ32 += nitems;
    } else if (have_x && !reused) {
      HPTRY(apply_op(c, kp, 1, nk, nb, c->X, c->AX, eps_items, rows));
      *happ64 += nitems;
    }
    ax_fresh = have_x && !ax32;
    HPCHK(launch_fill_int(c->count, kCntStep, 0, c->stream));
    HPCHK(timed(c, K_RESIDUAL64, [&] {
      if (ax32)
        return launch_residual64_ax32(kp, nb, nitems, c->B, c->AP32, c->R, c->B32, c->ld, c->d_npw, c->bn, c->rn,
                                      c->act_out, tol, c->count + kCntResid, c->floor_in, c->stream);
      return launch_residual64(kp, nb, nitems, c->B, c->AX, have_x, c->R, c->B32, c->ld, c->d_npw, c->bn, c->rn,
                               c->act_out, tol, c->count + kCntResid, c->floor_in, c->stream);
    }));
    HPCHK(hipMemcpyAsync(h_count, c->count, kCntStep * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HPTRY(sync(c));
    if (h_count[kCntResid + 1] > 0) return fail(HP_ERR_NUMERIC, "non-finite residual in the Sternheimer solve");
    nact = h_count[kCntResid];
    if (nact == 0 || ref == max_refine) break;
    // inner FP32 PCG on the refined items.  Its stopping threshold per item is
    // max(tol_in ||r0||, floor) with floor = tol ||B|| / 2 (set by the residual kernel).
    // When the inner result is trusted as the final one, the relative part is dropped
    // (tol_in = 0): the inner solve then runs to the outer tolerance itself, whatever
    // inner_tol is, so a cold start with tol < inner_tol is not stopped early.
    const double tol_in = trust ? 0.0 : inner_tol;
    HPCHK(timed(c, K_CG_INIT, [&] {
      return launch_cg_init32(kp, nb, nitems, c->B32, c->X32, c->R32, c->P32, c->d_diag, eps_items, c->ld, c->d_npw,
                              c->ld, c->rz_in, c->bn_in, c->rn_in, c->act_in, tol_in, c->act_out, c->floor_in,
                              c->stream);
    }));
    HPTRY(set_tol(c, 1, tol_in));
    int inner_active = nact;  // at most the refined items
    int k_in = 0;
    while (inner_active > 0 && k_in < max_it) {
      int steps = 0;
      long stepped = 0;
      HPTRY(cg_run_chunk(c, 1, chunk_len(c, 1, k_in, max_it), kp, nk, eps_items, inner_active, &steps, &stepped,
                         &inner_active));
      k_in += steps;
      *happ32 += stepped;
    }
    c->prev_iters[1] = k_in;
    it_in += k_in;
    HPCHK(timed(c, K_REFINE, [&] {
      return launch_refine_update(nb, nitems, c->X, c->X32, c->ld, c->act_out, have_x, c->stream);
    }));
    ax_fresh = false;
    // Above ~1e-6 the FP32 operator is exact enough that the inner solve's own residual
    // stands for the FP64 one; the next SCF iteration starts from an FP64 residual anyway.
    if (trust && inner_active == 0) {
      nact = 0;
      ++ref;
      trusted = true;
      break;
    }
  }
  c->ax_valid = ax_fresh;
  *iters = it_in;
  *refines = ref;
  *not_conv = nact;
  std::vector<double> rn(nitems), bn(nitems);
  // the last residual is the FP64 one, or the inner solve's when the FP32 result was trusted
  HPCHK(hipMemcpyAsync(rn.data(), trusted ? c->rn_in : c->rn, sizeof(double) * nitems, hipMemcpyDeviceToHost,
                       c->stream));
  HPCHK(hipMemcpyAsync(bn.data(), c->bn, sizeof(double) * nitems, hipMemcpyDeviceToHost, c->stream));
  HPTRY(sync(c));
  double m = 0.0;
  for (int i = 0; i < nitems; ++i)
    if (bn[i] > 0) m = std::max(m, rn[i] / bn[i]);
  *max_rel = m;
  return HP_OK;
}

hp_status upload_pairs(hp_ctx *c, int site, const double q[3], std::vector<KPair> &pairs) {
  (void)site;
  pairs.clear();
  for (int k = 0; k < c->n_mesh; ++k) {
    KPair P{};
    P.ek = k;
    P.ej = -1;
    P.spin = c->ent[k].spin;
    P.weight = c->ent[k].weight;
    for (int j = 0; j < c->n_kpts && P.ej < 0; ++j) {
      if (c->ent[j].spin != P.spin) continue;
      double d[3];
      bool ok = true;
      for (int a = 0; a < 3; ++a) {
        d[a] = c->ent[k].k[a] + q[a] - c->ent[j].k[a];
        if (std::fabs(d[a] - std::round(d[a])) > 1e-9) ok = false;
      }
      if (ok) {
        P.ej = j;
        for (int a = 0; a < 3; ++a) P.g0[a] = (int)std::lround(d[a]);
      }
    }
    if (P.ej < 0)
      return fail(HP_ERR_SHAPE, "no loaded entry holds k+q for mesh point %d, q = (%g, %g, %g)", k, q[0], q[1], q[2]);
    pairs.push_back(P);
  }
  // the largest shift of a k+q basis, for the plane variants that assume a bounded sphere
  for (int d = 0; d < 2; ++d) {
    int g = 0;
    for (const KPair &P : pairs) g = std::max(g, std::abs(P.g0[d]));
    c->pl.g0ext[d] = g;
    c->pl32.g0ext[d] = g;
  }
  HPCHK(hipMemcpyAsync(c->d_kp, pairs.data(), sizeof(KPair) * pairs.size(), hipMemcpyHostToDevice, c->stream));
  return HP_OK;
}

// Metallic ground state: per pair (k, k+q) the weights beta_ij = f_i theta_ij + f_j theta_ji +
// alpha theta_ji (f_i - f_j)/(e_i - e_j) of the projection onto the kept bands j of k+q
// (equal energies: the occupation derivative), stored [pair][j][i], and the occupations of
// the right-hand-side rows.
hp_status upload_metal(hp_ctx *c, const std::vector<KPair> &pairs) {
  const int nb = c->n_occ;
  const double sig = c->degauss;
  std::vector<double> beta((size_t)pairs.size() * nb * nb), focc((size_t)pairs.size() * nb);
  for (size_t k = 0; k < pairs.size(); ++k) {
    const double *fi = &c->occ_f[(size_t)pairs[k].ek * nb], *fj = &c->occ_f[(size_t)pairs[k].ej * nb];
    const double *ei = &c->ent_eps[(size_t)pairs[k].ek * nb], *ej = &c->ent_eps[(size_t)pairs[k].ej * nb];
    for (int i = 0; i < nb; ++i) {
      focc[k * nb + i] = fi[i];
      for (int j = 0; j < nb; ++j) {
        const double d = ei[i] - ej[j];
        const double th_ji = split_step(-d / sig);
        const double F = std::fabs(d) < 1e-9 ? -cold_delta((c->efermi - 0.5 * (ei[i] + ej[j])) / sig) / sig
                                             : (fi[i] - fj[j]) / d;
        beta[((size_t)k * nb + j) * nb + i] = fi[i] * (1.0 - th_ji) + fj[j] * th_ji + c->alpha * th_ji * F;
      }
    }
  }
  HPCHK(hipMemcpyAsync(c->d_beta, beta.data(), sizeof(double) * beta.size(), hipMemcpyHostToDevice, c->stream));
  HPCHK(hipMemcpyAsync(c->d_focc, focc.data(), sizeof(double) * focc.size(), hipMemcpyHostToDevice, c->stream));
  return sync(c);  // the host vectors go out of scope
}

// Small complex Hermitian solve (Gaussian elimination with partial pivoting).
bool csolve(int n, std::vector<std::complex<double>> A, std::vector<std::complex<double>> &b) {
  for (int i = 0; i < n; ++i) {
    int p = i;
    for (int r = i + 1; r < n; ++r)
      if (std::abs(A[r * n + i]) > std::abs(A[p * n + i])) p = r;
    if (std::abs(A[p * n + i]) == 0.0) return false;
    if (p != i) {
      for (int cc = 0; cc < n; ++cc) std::swap(A[i * n + cc], A[p * n + cc]);
      std::swap(b[i], b[p]);
    }
    for (int r = i + 1; r < n; ++r) {
      const std::complex<double> f = A[r * n + i] / A[i * n + i];
      for (int cc = i; cc < n; ++cc) A[r * n + cc] -= f * A[i * n + cc];
      b[r] -= f * b[i];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    std::complex<double> s = b[i];
    for (int cc = i + 1; cc < n; ++cc) s -= A[i * n + cc] * b[cc];
    b[i] = s / A[i * n + i];
  }
  return true;
}

hp_status zdots(hp_ctx *c, int nvec, const double2 *const *vecs, const double2 *b, long n,
                std::vector<std::complex<double>> &out) {
  HPCHK(hipMemcpyAsync(c->ptrs, vecs, sizeof(double2 *) * nvec, hipMemcpyHostToDevice, c->stream));
  HPCHK(timed(c, K_MIX, [&] {
    return launch_zdots(nvec, c->ptrs, b, n, c->dots_part, c->dots, c->stream);
  }));
  std::vector<double2> h(nvec);
  HPCHK(hipMemcpyAsync(h.data(), c->dots, sizeof(double2) * nvec, hipMemcpyDeviceToHost, c->stream));
  HPTRY(sync(c));
  out.resize(nvec);
  for (int i = 0; i < nvec; ++i) out[i] = {h[i].x, h[i].y};
  return HP_OK;
}

// Per-call controls that the kernels' launch paths read from the context.
void apply_call_params(hp_ctx *c, const hp_scf_params *p) {
  c->graph_chunk = p->graph_chunk;
  c->use_tuned = p->autotune;
  c->lowp_gemm = p->lowp_gemm;
}

// Ortho-atomic Hubbard projectors (Eq. 6) into c->d_phi: every entry's atomic orbitals in
// the stick order, their overlaps O_k on the matrix cores (one launch over all entries),
// O_k^-1/2 on the host (one thread per entry), then phi~_{5s+m} = sum_j (O^-1/2)_{j,r}
// phi_j with r = hub_rows[5s+m] on the matrix cores (one launch).
hp_status ortho_atomic_projectors(hp_ctx *c, const hp_ground_state *gs, const std::vector<const hp_kpoint *> &KP,
                                  const int *d_order, const std::vector<int> &pw_off) {
  const int na = gs->n_atwfc, nh5 = 5 * c->n_hub, ne = c->n_kpts;
  const long at_stride = (long)na * c->ld;
  const bool on_dev = gs->inputs_on_device == 1;
  const int ns = std::max(1, std::min(8, c->npw_max / 512));
  double2 *d_at = nullptr, *d_part = nullptr, *d_O = nullptr, *d_X = nullptr, *stage = nullptr;
  HPTRY(dalloc(&d_at, (size_t)ne * at_stride));
  hp_status st = HP_OK;
  auto cleanup = [&] {
    (void)hipStreamSynchronize(c->stream);
    for (double2 *ptr : {d_at, d_part, d_O, d_X, stage})
      if (ptr) (void)hipFree(ptr);
  };
  std::vector<std::complex<double>> O((size_t)ne * na * na), X((size_t)ne * na * nh5);
  do {
    if ((st = dalloc(&d_part, (size_t)ns * ne * na * na)) != HP_OK) break;
    if ((st = dalloc(&d_O, (size_t)ne * na * na)) != HP_OK) break;
    if ((st = dalloc(&d_X, (size_t)ne * na * nh5)) != HP_OK) break;
    if (!on_dev && (st = dalloc(&stage, (size_t)na * c->npw_max)) != HP_OK) break;
    // every entry's orbitals in the stick order (host arrays staged through one buffer)
    hipError_t e = hipSuccess;
    for (int i = 0; i < ne && e == hipSuccess; ++i) {
      const hp_kpoint &k = *KP[i];
      const double2 *from = (const double2 *)k.atwfc;
      if (!on_dev) {
        e = hipMemcpyAsync(stage, k.atwfc, sizeof(double2) * (size_t)na * k.npw, hipMemcpyHostToDevice, c->stream);
        from = stage;
      }
      if (e == hipSuccess) e = launch_gather_rows(from, k.npw, d_order + pw_off[i], na, d_at + (size_t)i * at_stride,
                                                  c->ld, c->stream);
      if (e == hipSuccess && !on_dev) e = hipStreamSynchronize(c->stream);
    }
    if (e == hipSuccess)
      e = launch_zproj(c->d_kself, 0, ne, d_at, at_stride, 0, na, d_at, c->ld, na, c->d_npw, d_part, ns, nullptr, 0,
                       c->stream);
    if (e == hipSuccess) e = launch_zproj_reduce(ne, na, na, ns, d_part, nullptr, 1.0, d_O, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(O.data(), d_O, sizeof(double2) * O.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      st = fail(HP_ERR_HIP, "ortho-atomic overlaps: %s", hipGetErrorString(e));
      break;
    }
    // O^-1/2 per entry; keep the columns of the Hubbard rows: X[e][j][v] = (O^-1/2)_{j, hub_rows[v]}
    std::vector<int> bad(ne, 0);
    const int nthreads = std::max(1, std::min(ne, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t)
      pool.emplace_back([&, t] {
        std::vector<std::complex<double>> full((size_t)na * na);
        for (int i = t; i < ne; i += nthreads) {
          if (!inv_sqrt_hermitian(na, O.data() + (size_t)i * na * na, full.data())) {
            bad[i] = 1;
            continue;
          }
          for (int j = 0; j < na; ++j)
            for (int v = 0; v < nh5; ++v)
              X[((size_t)i * na + j) * nh5 + v] = full[(size_t)j * na + gs->hub_rows[v]];
        }
      });
    for (auto &th : pool) th.join();
    for (int i = 0; i < ne; ++i)
      if (bad[i]) {
        st = fail(HP_ERR_SINGULAR, "kpts[%d]: atomic orbitals are linearly dependent", i);
        break;
      }
    if (st != HP_OK) break;
    e = hipMemcpyAsync(d_X, X.data(), sizeof(double2) * X.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(c->d_phi, 0, sizeof(double2) * (size_t)ne * c->phi_stride, c->stream);
    if (e == hipSuccess)
      e = launch_zexpand(c->d_kself, 0, ne, d_at, at_stride, 0, na, d_X, (long)na * nh5, 1.0, c->d_phi, c->ld, nh5,
                         c->d_npw, c->npw_max, nullptr, 1, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = fail(HP_ERR_HIP, "ortho-atomic projectors: %s", hipGetErrorString(e));
  } while (false);
  cleanup();
  return st;
}

hp_status check_params(const hp_scf_params *p) {
  if (!p) return fail(HP_ERR_ARG, "params is NULL");
  if (p->struct_size != sizeof(hp_scf_params)) return fail(HP_ERR_ARG, "hp_scf_params.struct_size mismatch");
  if (!(p->cg_tol > 0.0) || !(p->conv_thr_chi > 0.0) || !(p->conv_thr_v > 0.0))
    return fail(HP_ERR_ARG, "thresholds must be positive");
  if (p->niter_max < 1 || p->max_cg_iter < 1) return fail(HP_ERR_ARG, "iteration limits must be >= 1");
  if (p->nmix < 1 || p->nmix > kNmixMax) return fail(HP_ERR_ARG, "nmix must be in 1..%d", kNmixMax);
  if (!(p->alpha_mix > 0.0 && p->alpha_mix <= 1.0)) return fail(HP_ERR_ARG, "alpha_mix must be in (0, 1]");
  if (p->precision != HP_FP64 && p->precision != HP_MIXED) return fail(HP_ERR_ARG, "unknown precision %d", p->precision);
  if (p->precision == HP_MIXED && (!(p->inner_tol > 0.0 && p->inner_tol < 1.0) || p->max_refine < 1))
    return fail(HP_ERR_ARG, "inner_tol must be in (0, 1) and max_refine >= 1");
  if (p->graph_chunk < 0 || p->graph_chunk > kMaxChunk)
    return fail(HP_ERR_ARG, "graph_chunk must be in 0..%d", kMaxChunk);
  if (p->autotune != 0 && p->autotune != 1) return fail(HP_ERR_ARG, "autotune must be 0 or 1");
  if (p->lowp_gemm < HP_GEMM_FP32 || p->lowp_gemm > HP_GEMM_BF16_PV32)
    return fail(HP_ERR_ARG, "unknown lowp_gemm %d", p->lowp_gemm);
  if (p->skip_equivalence_q != 0 && p->skip_equivalence_q != 1)
    return fail(HP_ERR_ARG, "skip_equivalence_q must be 0 or 1");
  if (p->find_atpert != 0 && p->find_atpert != 1 && p->find_atpert != 4)
    return fail(HP_ERR_ARG, "find_atpert must be 1 or 4 (0 = 4)");
  if (p->find_atpert == 1 && (!(p->docc_thr >= 0.0) || !(p->dist_thr >= 0.0)))
    return fail(HP_ERR_ARG, "docc_thr and dist_thr must be >= 0");
  if (!(p->lowp_trust_tol >= 0.0)) return fail(HP_ERR_ARG, "lowp_trust_tol must be >= 0 (0: the default 1e-6)");
  return HP_OK;
}

// Ground-state occupation trace (summed over spins) and moment of every Hubbard site (Eq. 3)
// from the projections A_k[m][v] = <phi_{m,k}|u_vk> of the mesh entries.
hp_status site_occupations(hp_ctx *c, std::vector<double> &trace, std::vector<double> &moment) {
  const int nb = c->n_occ, M = 5 * c->n_hub;
  std::vector<double2> A((size_t)c->n_mesh * M * nb);
  HPCHK(hipMemcpyAsync(A.data(), c->d_A, sizeof(double2) * A.size(), hipMemcpyDeviceToHost, c->stream));
  HPTRY(sync(c));
  std::vector<double> per_spin((size_t)2 * c->n_hub, 0.0);
  for (int k = 0; k < c->n_mesh; ++k) {
    const double w = c->occ * c->ent[k].weight;
    for (int s2 = 0; s2 < c->n_hub; ++s2) {
      double t = 0.0;
      for (int m = 0; m < 5; ++m)
        for (int v = 0; v < nb; ++v) {  // weighted by the band occupation (1 for insulators)
          const double2 a = A[((size_t)k * M + 5 * s2 + m) * nb + v];
          t += c->occ_f[(size_t)k * nb + v] * (a.x * a.x + a.y * a.y);
        }
      per_spin[(size_t)c->ent[k].spin * c->n_hub + s2] += w * t;
    }
  }
  trace.assign(c->n_hub, 0.0);
  moment.assign(c->n_hub, 0.0);
  for (int s2 = 0; s2 < c->n_hub; ++s2) {
    trace[s2] = per_spin[s2] + per_spin[c->n_hub + s2];
    if (c->nspin == 2) moment[s2] = per_spin[s2] - per_spin[c->n_hub + s2];
  }
  return HP_OK;
}

// Representative of every site: the first earlier representative whose trace is within thr.
std::vector<int> site_classes(const std::vector<double> &trace, double thr) {
  std::vector<int> rep(trace.size());
  for (size_t s2 = 0; s2 < trace.size(); ++s2) {
    rep[s2] = (int)s2;
    for (size_t u = 0; u < s2; ++u)
      if (rep[u] == (int)u && std::fabs(trace[u] - trace[s2]) < thr) {
        rep[s2] = (int)u;
        break;
      }
  }
  return rep;
}

// Minimum-image distances between all sites of the q-supercell (index l * n_hub + s, cells l
// lexicographic with the last index fastest), over supercell translations two shells out.
std::vector<double> supercell_distances(const double cell[9], int n_hub, const double *hub_tau, const int nq[3]) {
  const int nc = nq[0] * nq[1] * nq[2], n = n_hub * nc;
  std::vector<std::array<double, 3>> pos(n);
  for (int a = 0, l = 0; a < nq[0]; ++a)
    for (int b = 0; b < nq[1]; ++b)
      for (int d = 0; d < nq[2]; ++d, ++l)
        for (int s2 = 0; s2 < n_hub; ++s2)
          for (int x = 0; x < 3; ++x)
            pos[l * n_hub + s2][x] = hub_tau[3 * s2 + x] + a * cell[x] + b * cell[3 + x] + d * cell[6 + x];
  std::vector<double> D((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double best = 1e300;
      for (int u = -2; u <= 2; ++u)
        for (int v = -2; v <= 2; ++v)
          for (int w = -2; w <= 2; ++w) {
            double r2 = 0.0;
            for (int x = 0; x < 3; ++x) {
              const double t = u * nq[0] * cell[x] + v * nq[1] * cell[3 + x] + w * nq[2] * cell[6 + x];
              const double dx = pos[j][x] - pos[i][x] + t;
              r2 += dx * dx;
            }
            best = std::min(best, r2);
          }
      D[(size_t)i * n + j] = std::sqrt(best);
    }
  return D;
}

}  // namespace

// =============================================================== ABI

extern "C" const char *hp_last_error(void) { return g_err.c_str(); }

extern "C" void hp_destroy(hp_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  for (void *p : c->allocs) (void)hipFree(p);
  for (auto &p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < 16; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" hp_status hp_neighbours(const double cell[9], int32_t n_hub, const double *hub_tau, const int32_t nq[3],
                                   double dist_thr, int32_t max_pairs, int32_t *pair_i, int32_t *pair_j, double *dist,
                                   int32_t *n_pairs) {
  if (!cell || !hub_tau || !nq || !n_pairs || (max_pairs > 0 && (!pair_i || !pair_j || !dist)))
    return fail(HP_ERR_ARG, "NULL argument");
  if (n_hub < 1 || nq[0] < 1 || nq[1] < 1 || nq[2] < 1 || !(dist_thr >= 0.0))
    return fail(HP_ERR_ARG, "need n_hub >= 1, nq >= 1, dist_thr >= 0");
  const int nc = nq[0] * nq[1] * nq[2], n = n_hub * nc;
  const std::vector<double> D = supercell_distances(cell, n_hub, hub_tau, nq);
  auto min_image = [&](int i, int j) { return D[(size_t)i * n + j]; };
  int found = 0;
  for (int i = 0; i < n_hub; ++i) {
    std::vector<double> dj(n, 0.0);
    double dmin = 1e300;
    for (int j = 0; j < n; ++j)
      if (j != i) {
        dj[j] = min_image(i, j);
        dmin = std::min(dmin, dj[j]);
      }
    for (int j = 0; j < n; ++j)
      if (j != i && dj[j] <= dmin + dist_thr) {
        if (found < max_pairs) {
          pair_i[found] = i;
          pair_j[found] = j;
          dist[found] = dj[j];
        }
        ++found;
      }
  }
  *n_pairs = found;
  if (found > max_pairs) return fail(HP_ERR_ARG, "%d pairs found, max_pairs = %d", found, max_pairs);
  return HP_OK;
}

extern "C" hp_status hp_hubbard_params(int32_t n, const double *chi0, const double *chi, double *uv_out) {
  if (n < 1) return fail(HP_ERR_ARG, "n = %d", n);
  if (!chi0 || !chi || !uv_out) return fail(HP_ERR_ARG, "NULL argument");
  std::vector<double> inv0, inv1;
  for (int which = 0; which < 2; ++which) {
    const double *M = which == 0 ? chi0 : chi;
    double amax = 0.0;
    for (long i = 0; i < (long)n * n; ++i) {
      if (!std::isfinite(M[i])) return fail(HP_ERR_NUMERIC, "non-finite entry in %s", which ? "chi" : "chi0");
      amax = std::max(amax, std::fabs(M[i]));
    }
    if (amax == 0.0) return fail(HP_ERR_SINGULAR, "%s is zero", which ? "chi" : "chi0");
    // Gauss-Jordan inversion with partial pivoting, FP64
    std::vector<double> A(M, M + (long)n * n), I((long)n * n, 0.0);
    for (int i = 0; i < n; ++i) I[(long)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
      int p = col;
      for (int r = col + 1; r < n; ++r)
        if (std::fabs(A[(long)r * n + col]) > std::fabs(A[(long)p * n + col])) p = r;
      if (std::fabs(A[(long)p * n + col]) < 1e-14 * amax)
        return fail(HP_ERR_SINGULAR, "%s is singular (pivot %g)", which ? "chi" : "chi0", A[(long)p * n + col]);
      if (p != col)
        for (int cc = 0; cc < n; ++cc) {
          std::swap(A[(long)p * n + cc], A[(long)col * n + cc]);
          std::swap(I[(long)p * n + cc], I[(long)col * n + cc]);
        }
      const double d = A[(long)col * n + col];
      for (int cc = 0; cc < n; ++cc) {
        A[(long)col * n + cc] /= d;
        I[(long)col * n + cc] /= d;
      }
      for (int r = 0; r < n; ++r) {
        if (r == col) continue;
        const double f = A[(long)r * n + col];
        if (f == 0.0) continue;
        for (int cc = 0; cc < n; ++cc) {
          A[(long)r * n + cc] -= f * A[(long)col * n + cc];
          I[(long)r * n + cc] -= f * I[(long)col * n + cc];
        }
      }
    }
    (which == 0 ? inv0 : inv1) = I;
  }
  for (long i = 0; i < (long)n * n; ++i) uv_out[i] = inv0[i] - inv1[i];
  return HP_OK;
}

extern "C" hp_status hp_ground_state_load(const hp_ground_state *gs, hp_ctx **out) {
  if (!out) return fail(HP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!gs) return fail(HP_ERR_ARG, "gs is NULL");
  if (gs->struct_size != sizeof(hp_ground_state)) return fail(HP_ERR_ARG, "hp_ground_state.struct_size mismatch");
  if (gs->nspin != 1 && gs->nspin != 2) return fail(HP_ERR_ARG, "nspin must be 1 or 2");
  if (!(gs->degauss >= 0.0) || !std::isfinite(gs->degauss) || !std::isfinite(gs->efermi))
    return fail(HP_ERR_ARG, "degauss must be >= 0 and efermi finite");
  if (gs->degauss > 0.0 && gs->nspin != 1) return fail(HP_ERR_ARG, "metallic ground states must be unpolarized");
  if (gs->spin_factor != 3 - gs->nspin)
    return fail(HP_ERR_ARG, "spin_factor must be %d with nspin = %d", 3 - gs->nspin, gs->nspin);
  if (gs->xc != HP_XC_LDA_PZ81) return fail(HP_ERR_ARG, "unknown xc %d", gs->xc);
  if (gs->inputs_on_device != 0 && gs->inputs_on_device != 1) return fail(HP_ERR_ARG, "inputs_on_device must be 0 or 1");
  const bool on_dev = gs->inputs_on_device == 1;
  if (gs->projectors != HP_PROJ_ATOMIC && gs->projectors != HP_PROJ_ORTHO_ATOMIC)
    return fail(HP_ERR_ARG, "unknown projectors %d", gs->projectors);
  if (!gs->v_loc || !gs->rho0 || !gs->d_kb || !gs->hub_tau || !gs->kpts) return fail(HP_ERR_ARG, "NULL array");
  if (gs->n_occ < 1 || gs->n_beta < 0 || gs->n_hub < 1) return fail(HP_ERR_ARG, "bad n_occ/n_beta/n_hub");
  if (gs->projectors == HP_PROJ_ORTHO_ATOMIC) {
    if (gs->n_atwfc < 5 * gs->n_hub || !gs->hub_rows) return fail(HP_ERR_ARG, "need n_atwfc >= 5 n_hub and hub_rows");
    std::vector<char> seen(gs->n_atwfc, 0);
    for (int v = 0; v < 5 * gs->n_hub; ++v) {
      const int r = gs->hub_rows[v];
      if (r < 0 || r >= gs->n_atwfc || seen[r]) return fail(HP_ERR_ARG, "hub_rows[%d] = %d invalid or repeated", v, r);
      seen[r] = 1;
    }
  }
  if (gs->n_mesh < 1 || gs->n_kpts % gs->nspin || gs->n_kpts / gs->nspin < gs->n_mesh)
    return fail(HP_ERR_ARG, "bad n_mesh/n_kpts");
  std::vector<int> rad[3];
  for (int d = 0; d < 3; ++d) {
    if (gs->fft[d] < 2 || gs->fft[d] > 256 || !factor_235(gs->fft[d], rad[d]))
      return fail(HP_ERR_SHAPE, "fft[%d] = %d is not a product of 2, 3, 5 in [2, 256]", d, gs->fft[d]);
  }
  for (int i = 0; i < gs->n_kpts; ++i) HPTRY(check_kpoint(gs->kpts[i], i, gs));
  // spin blocks: the same k points and spheres in the same order
  const int nks = gs->n_kpts / gs->nspin;
  for (int i = 0; gs->nspin == 2 && i < nks; ++i) {
    const hp_kpoint &a = gs->kpts[i], &b = gs->kpts[nks + i];
    bool same = a.npw == b.npw;
    for (int d = 0; d < 3 && same; ++d) same = a.k_frac[d] == b.k_frac[d];
    for (long j = 0; j < 3L * a.npw && same; ++j) same = a.miller[j] == b.miller[j];
    if (!same) return fail(HP_ERR_ARG, "kpts[%d] (spin down) differs from kpts[%d] in k or sphere", nks + i, i);
  }
  // internal order: mesh entries of every spin, then the extra k+q entries of every spin
  std::vector<const hp_kpoint *> KP;
  std::vector<int> internal_of(gs->n_kpts), spin_of;
  for (int pass = 0; pass < 2; ++pass)
    for (int sp = 0; sp < gs->nspin; ++sp)
      for (int i = pass ? gs->n_mesh : 0; i < (pass ? nks : gs->n_mesh); ++i) {
        internal_of[sp * nks + i] = (int)KP.size();
        KP.push_back(&gs->kpts[sp * nks + i]);
        spin_of.push_back(sp);
      }
  const double det = gs->cell[0][0] * (gs->cell[1][1] * gs->cell[2][2] - gs->cell[1][2] * gs->cell[2][1]) -
                     gs->cell[0][1] * (gs->cell[1][0] * gs->cell[2][2] - gs->cell[1][2] * gs->cell[2][0]) +
                     gs->cell[0][2] * (gs->cell[1][0] * gs->cell[2][1] - gs->cell[1][1] * gs->cell[2][0]);
  if (!(std::fabs(det) > 1e-8)) return fail(HP_ERR_ARG, "degenerate cell");
  // plane-wave layouts (host), before any GPU call
  std::vector<Layout> lay(gs->n_kpts);
  for (int i = 0; i < gs->n_kpts; ++i)
    HPTRY(build_layout(*KP[i], gs->fft[0], gs->fft[1], gs->fft[2], lay[i], i));
  for (int i = 0; i < gs->n_kpts; ++i) {
    const hp_kpoint &k = *KP[i];
    for (int v = 0; v < gs->n_occ; ++v)
      if (!std::isfinite(k.eps[v])) return fail(HP_ERR_NUMERIC, "kpts[%d].eps[%d] is not finite", i, v);
  }
  // ground-state Hubbard potential: finite, Hermitian per (spin, site); its eigenpairs give
  // the projector rows that carry it (sum_a lam_a |chi_a><chi_a|, chi_a = sum_m V_ma phi_m)
  std::vector<double> hub_lam;
  std::vector<std::complex<double>> hub_vec;
  if (gs->hub_pot) {
    const int nblk = gs->nspin * gs->n_hub;
    hub_lam.resize((size_t)nblk * 5);
    hub_vec.resize((size_t)nblk * 25);
    for (int b = 0; b < nblk; ++b) {
      std::complex<double> M[25];
      double big = 0.0;
      for (int i = 0; i < 25; ++i) {
        M[i] = {gs->hub_pot[2 * (25 * b + i)], gs->hub_pot[2 * (25 * b + i) + 1]};
        if (!std::isfinite(M[i].real()) || !std::isfinite(M[i].imag()))
          return fail(HP_ERR_NUMERIC, "hub_pot block %d is not finite", b);
        big = std::max(big, std::abs(M[i]));
      }
      for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j)
          if (std::abs(M[i * 5 + j] - std::conj(M[j * 5 + i])) > 1e-10 * (1.0 + big))
            return fail(HP_ERR_ARG, "hub_pot block %d (spin %d, site %d) is not Hermitian", b, b / gs->n_hub,
                        b % gs->n_hub);
      if (!herm_eig(5, M, hub_lam.data() + 5 * b, hub_vec.data() + 25 * b))
        return fail(HP_ERR_NUMERIC, "hub_pot block %d: eigen-decomposition failed", b);
    }
  }
  const long nrr = (long)gs->fft[0] * gs->fft[1] * gs->fft[2] * gs->nspin;
  if (!on_dev)  // device inputs are checked on the device below
    for (long i = 0; i < nrr; ++i)
      if (!std::isfinite(gs->v_loc[i]) || !std::isfinite(gs->rho0[i])) return fail(HP_ERR_NUMERIC, "non-finite v_loc/rho0");

  // on an early error return the partly built context, device memory included, is destroyed
  std::unique_ptr<hp_ctx, void (*)(hp_ctx *)> c(new hp_ctx(), hp_destroy);
  for (int i = 0; i < 16; ++i) c->ev[i] = nullptr;
  c->n1 = gs->fft[0];
  c->n2 = gs->fft[1];
  c->n3 = gs->fft[2];
  c->np = (long)c->n1 * c->n2;
  c->nr = c->np * c->n3;
  c->n_occ = gs->n_occ;
  // the stacked table holds the KB rows, then (with a ground-state Hubbard potential) 5 n_hub
  // rows of scale +1 and 5 n_hub rows of scale -1 that carry it, then the occupied states
  c->n_kb = gs->n_beta;
  c->n_beta = gs->n_beta + (gs->hub_pot ? 10 * gs->n_hub : 0);
  c->n_hub = gs->n_hub;
  c->nspin = gs->nspin;
  c->n_mesh_spin = gs->n_mesh;
  c->n_mesh = gs->nspin * gs->n_mesh;
  c->occ = gs->nspin == 2 ? 1.0 : 2.0;
  c->internal_of = internal_of;
  c->degauss = gs->degauss;
  c->efermi = gs->efermi;
  c->ent_eps.resize((size_t)gs->n_kpts * gs->n_occ);
  c->occ_f.assign(c->ent_eps.size(), 1.0);
  c->occ_d.assign(c->ent_eps.size(), 0.0);
  for (int i = 0; i < gs->n_kpts; ++i)
    for (int v = 0; v < gs->n_occ; ++v) {
      const double e = KP[i]->eps[v];
      c->ent_eps[(size_t)i * gs->n_occ + v] = e;
      if (gs->degauss > 0.0) {
        c->occ_f[(size_t)i * gs->n_occ + v] = cold_occ((gs->efermi - e) / gs->degauss);
        c->occ_d[(size_t)i * gs->n_occ + v] = cold_delta((gs->efermi - e) / gs->degauss);
      }
    }
  c->n_kpts = gs->n_kpts;
  c->n_proj = c->n_beta + c->n_occ;
  for (int i = 0; i < 9; ++i) c->cell[i] = gs->cell[i / 3][i % 3];
  c->hub_tau.assign(gs->hub_tau, gs->hub_tau + 3 * gs->n_hub);
  c->omega = std::fabs(det);
  {
    // b = 2 pi inv(A)^T: rows b_i with a_i . b_j = 2 pi delta_ij
    const double *a = c->cell;
    double inv[9];
    inv[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    inv[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    inv[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    inv[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    inv[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    inv[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    inv[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    inv[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    inv[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) c->bvec[i * 3 + j] = 2.0 * M_PI * inv[j * 3 + i];
  }
  // alpha = 2 (max - min) over the occupied energies of every entry (text after Eq. 18)
  double emax = -1e300, emin = 1e300;
  for (int i = 0; i < gs->n_kpts; ++i)
    for (int v = 0; v < gs->n_occ; ++v) {
      emax = std::max(emax, KP[i]->eps[v]);
      emin = std::min(emin, KP[i]->eps[v]);
    }
  c->alpha = std::max(2.0 * (emax - emin), 0.01);

  int npw_max = 0, ns_max = 0, chunk_max = 0;
  for (int i = 0; i < gs->n_kpts; ++i) {
    npw_max = std::max(npw_max, KP[i]->npw);
    const int ns = (int)lay[i].sx.size();
    ns_max = std::max(ns_max, ns);
    for (int s0 = 0; s0 < ns; s0 += 32) {
      const int s1 = std::min(s0 + 32, ns);
      chunk_max = std::max(chunk_max, lay[i].sstart[s1 - 1] + lay[i].slen[s1 - 1] - lay[i].sstart[s0]);
    }
  }
  int pw256 = 0;  // most plane waves in 256 consecutive sticks (LDS of the staged z transforms)
  for (int i = 0; i < gs->n_kpts; ++i) {
    const int ns = (int)lay[i].sx.size();
    for (int s0 = 0; s0 < ns; s0 += 256) {
      const int s1 = std::min(s0 + 256, ns);
      pw256 = std::max(pw256, lay[i].sstart[s1 - 1] + lay[i].slen[s1 - 1] - lay[i].sstart[s0]);
    }
  }
  c->npw_max = npw_max;
  c->ld = (npw_max + 63) / 64 * 64;
  c->ns_max = ns_max;
  c->ns_pad = (ns_max + 31) / 32 * 32;
  c->max_chunk_pw = chunk_max;
  c->t_stride = (long)c->n_proj * c->ld;
  c->phi_stride = (long)5 * c->n_hub * c->ld;

  // -------- device from here on
  if (gs->stream) {
    c->stream = (hipStream_t)gs->stream;
  } else {
    HPCHK(hipStreamCreate(&c->stream));
    c->own_stream = true;
  }
  hipStream_t st = c->stream;
  for (int i = 0; i < 16; ++i) HPCHK(hipEventCreate(&c->ev[i]));
  HPTRY(noalloc_scratch(&c->scratch));

  // FFT axes: twiddles and permutations
  const int N[3] = {c->n1, c->n2, c->n3};
  std::vector<double2> tw_h;
  int tw_off[3];
  for (int d = 0; d < 3; ++d) {
    tw_off[d] = (int)tw_h.size();
    for (int j = 0; j < N[d]; ++j)
      tw_h.push_back(make_double2(std::cos(2.0 * M_PI * j / N[d]), std::sin(2.0 * M_PI * j / N[d])));
  }
  HPTRY(c->alloc(&c->tw, tw_h.size()));
  HPCHK(hipMemcpyAsync(c->tw, tw_h.data(), sizeof(double2) * tw_h.size(), hipMemcpyHostToDevice, st));
  Axis ax[3];
  for (int d = 0; d < 3; ++d) {
    ax[d] = Axis{};
    ax[d].n = N[d];
    ax[d].nst = (int)rad[d].size();
    int pr = 1;
    for (int s = 0; s < ax[d].nst; ++s) {
      ax[d].rad[s] = rad[d][s];
      pr *= rad[d][s];
      ax[d].span[s] = N[d] / pr;
    }
    ax[d].tw = c->tw + tw_off[d];
  }
  c->pl.ax = ax[0];
  c->pl.ay = ax[1];
  c->pl.n1 = c->n1;
  c->pl.n2 = c->n2;
  c->pl.n3 = c->n3;
  c->pl.nxa_max = 0;
  c->pl.mext[0] = c->pl.mext[1] = 0;
  c->pl.g0ext[0] = c->pl.g0ext[1] = 0;
  for (int i = 0; i < gs->n_kpts; ++i) {
    c->pl.nxa_max = std::max(c->pl.nxa_max, (int)lay[i].xa.size());
    for (int d = 0; d < 2; ++d) c->pl.mext[d] = std::max(c->pl.mext[d], lay[i].mext[d]);
  }
  c->az = ax[2];
  if (c->np * (long)sizeof(double2) > 160 * 1024) return fail(HP_ERR_SHAPE, "xy plane does not fit in LDS");
  c->px = dif_perm(c->n1, rad[0]);
  c->py = dif_perm(c->n2, rad[1]);
  HPTRY(c->alloc(&c->d_px, c->n1));
  HPTRY(c->alloc(&c->d_py, c->n2));
  HPCHK(hipMemcpyAsync(c->d_px, c->px.data(), sizeof(int) * c->n1, hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(c->d_py, c->py.data(), sizeof(int) * c->n2, hipMemcpyHostToDevice, st));

  // local potential and f_xc in the permuted real-space layout
  // (per spin: [nspin][nr]; the kernel: [nr] unpolarized, [3][nr] = f_uu, f_ud, f_dd polarized)
  const int ns = c->nspin;
  double *d_nat = nullptr;
  HPTRY(c->alloc(&d_nat, (size_t)ns * c->nr));
  HPTRY(c->alloc(&c->d_vp, (size_t)ns * c->nr));
  HPTRY(c->alloc(&c->d_fxc, (size_t)(ns == 2 ? 3 : 1) * c->nr));
  // host inputs are copied in, device inputs (inputs_on_device) copied device to device
  const hipMemcpyKind in_kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  // per spin: sum and non-finite count of v_loc, then of rho0 (fixed-order reduction, so
  // host and device inputs give the same mean potential)
  double *d_stats = nullptr, *d_vmean = nullptr;
  HPTRY(c->alloc(&d_stats, (size_t)4 * ns));
  HPTRY(c->alloc(&d_vmean, 2));
  HPCHK(hipMemcpyAsync(d_nat, gs->v_loc, sizeof(double) * ns * c->nr, in_kind, st));
  HPCHK(launch_block_stats(d_nat, ns, c->nr, d_stats, st));
  for (int sp = 0; sp < ns; ++sp)
    HPCHK(launch_permute_real(c->pl, c->d_px, c->d_py, d_nat + sp * c->nr, c->d_vp + sp * c->nr, st));
  HPTRY(sync(c.get()));
  HPCHK(hipMemcpyAsync(d_nat, gs->rho0, sizeof(double) * ns * c->nr, in_kind, st));
  HPCHK(launch_block_stats(d_nat, ns, c->nr, d_stats + 2 * ns, st));
  double *d_rhop = nullptr;
  HPTRY(c->alloc(&d_rhop, (size_t)ns * c->nr));
  for (int sp = 0; sp < ns; ++sp)
    HPCHK(launch_permute_real(c->pl, c->d_px, c->d_py, d_nat + sp * c->nr, d_rhop + sp * c->nr, st));
  if (ns == 2)
    HPCHK(launch_fxc_spin(d_rhop, d_rhop + c->nr, c->d_fxc, c->nr, st));
  else
    HPCHK(launch_fxc(d_rhop, c->d_fxc, c->nr, st));
  HPTRY(c->alloc(&c->d_bvec, 9));
  HPCHK(hipMemcpyAsync(c->d_bvec, c->bvec, sizeof(double) * 9, hipMemcpyHostToDevice, st));
  double vmean_s[2] = {0.0, 0.0};
  {
    double h_stats[8];
    HPCHK(hipMemcpyAsync(h_stats, d_stats, sizeof(double) * 4 * ns, hipMemcpyDeviceToHost, st));
    HPTRY(sync(c.get()));
    for (int b = 0; b < 2 * ns; ++b)
      if (h_stats[2 * b + 1] != 0.0) return fail(HP_ERR_NUMERIC, "non-finite v_loc/rho0");
    for (int sp = 0; sp < ns; ++sp) vmean_s[sp] = h_stats[2 * sp] / (double)c->nr;
    HPCHK(hipMemcpyAsync(d_vmean, vmean_s, sizeof(double) * 2, hipMemcpyHostToDevice, st));
  }

  // per-entry tables in the stick order
  std::vector<int> h_sx, h_sy, h_ss, h_sl, h_iz, h_xa, h_npw(c->n_kpts), h_order;
  std::vector<EntryDev> h_ent(c->n_kpts);
  std::vector<double> h_kin;
  int pw_off = 0;
  c->ent.resize(c->n_kpts);
  for (int i = 0; i < c->n_kpts; ++i) {
    const hp_kpoint &k = *KP[i];
    const Layout &L = lay[i];
    EntryDev E{};
    E.npw = k.npw;
    E.ns = (int)L.sx.size();
    E.nxa = (int)L.xa.size();
    E.pw_off = pw_off;
    E.st_off = (int)h_sx.size();
    E.xa_off = (int)h_xa.size();
    h_ent[i] = E;
    h_npw[i] = k.npw;
    h_sx.insert(h_sx.end(), L.sx.begin(), L.sx.end());
    h_sy.insert(h_sy.end(), L.sy.begin(), L.sy.end());
    h_ss.insert(h_ss.end(), L.sstart.begin(), L.sstart.end());
    h_sl.insert(h_sl.end(), L.slen.begin(), L.slen.end());
    h_iz.insert(h_iz.end(), L.iz.begin(), L.iz.end());
    h_xa.insert(h_xa.end(), L.xa.begin(), L.xa.end());
    pw_off += k.npw;
    HostEntry &he = c->ent[i];
    for (int a = 0; a < 3; ++a) he.k[a] = k.k_frac[a];
    he.weight = k.weight;
    he.npw = k.npw;
    he.spin = spin_of[i];
    he.order = L.order;
    he.pw_off = E.pw_off;
    h_order.insert(h_order.end(), L.order.begin(), L.order.end());
    for (int p = 0; p < k.npw; ++p) {
      const int q = L.order[p];
      double kv[3];
      for (int a = 0; a < 3; ++a) {
        kv[a] = 0.0;
        for (int b = 0; b < 3; ++b) kv[a] += (k.miller[3 * q + b] + k.k_frac[b]) * c->bvec[b * 3 + a];
      }
      h_kin.push_back(0.5 * (kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2]));
    }
  }
  int *d_sx, *d_sy, *d_ss, *d_sl, *d_iz, *d_xa;
  EntryDev *d_ent;
  HPTRY(c->alloc(&d_sx, h_sx.size()));
  HPTRY(c->alloc(&d_sy, h_sy.size()));
  HPTRY(c->alloc(&d_ss, h_ss.size()));
  HPTRY(c->alloc(&d_sl, h_sl.size()));
  HPTRY(c->alloc(&d_iz, h_iz.size()));
  HPTRY(c->alloc(&d_xa, h_xa.size()));
  HPTRY(c->alloc(&d_ent, h_ent.size()));
  HPTRY(c->alloc(&c->d_npw, h_npw.size()));
  HPTRY(c->alloc(&c->d_kin, h_kin.size()));
  HPTRY(c->alloc(&c->d_diag, (size_t)c->n_kpts * c->ld));
  HPTRY(c->alloc(&c->d_T, (size_t)c->n_kpts * c->t_stride));
  HPTRY(c->alloc(&c->d_phi, (size_t)c->n_kpts * c->phi_stride));
  int *d_order = nullptr;
  HPTRY(c->alloc(&d_order, h_order.size()));
  c->d_order = d_order;
  HPCHK(hipMemcpyAsync(d_sx, h_sx.data(), sizeof(int) * h_sx.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(d_sy, h_sy.data(), sizeof(int) * h_sy.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(d_ss, h_ss.data(), sizeof(int) * h_ss.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(d_sl, h_sl.data(), sizeof(int) * h_sl.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(d_iz, h_iz.data(), sizeof(int) * h_iz.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(d_xa, h_xa.data(), sizeof(int) * h_xa.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(d_ent, h_ent.data(), sizeof(EntryDev) * h_ent.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(c->d_npw, h_npw.data(), sizeof(int) * h_npw.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(c->d_kin, h_kin.data(), sizeof(double) * h_kin.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemcpyAsync(d_order, h_order.data(), sizeof(int) * h_order.size(), hipMemcpyHostToDevice, st));
  HPCHK(hipMemsetAsync(c->d_T, 0, sizeof(double2) * (size_t)c->n_kpts * c->t_stride, st));
  HPCHK(hipMemsetAsync(c->d_phi, 0, sizeof(double2) * (size_t)c->n_kpts * c->phi_stride, st));
  {
    // KB rows, occupied states and (atomic projectors) the d orbitals of every entry, gathered
    // into the stick order on the device: from the caller's device arrays, or from host
    // arrays staged through one device buffer
    const int nphi = gs->projectors == HP_PROJ_ATOMIC ? 5 * c->n_hub : 0;
    const int nrow = c->n_kb + c->n_occ + nphi;
    double2 *stage = nullptr;
    if (!on_dev) HPTRY(dalloc(&stage, (size_t)nrow * c->npw_max));
    hp_status sst = HP_OK;
    for (int i = 0; i < c->n_kpts && sst == HP_OK; ++i) {
      const hp_kpoint &k = *KP[i];
      const int npw = k.npw;
      const int *ord = d_order + h_ent[i].pw_off;
      const double2 *src[3] = {(const double2 *)k.beta, (const double2 *)k.u, (const double2 *)k.phi};
      const int rows[3] = {c->n_kb, c->n_occ, nphi};
      double2 *dst[3] = {c->d_T + (size_t)i * c->t_stride, c->d_T + (size_t)i * c->t_stride + (size_t)c->n_beta * c->ld,
                         c->d_phi + (size_t)i * c->phi_stride};
      size_t off = 0;
      hipError_t e = hipSuccess;
      for (int t = 0; t < 3 && e == hipSuccess; ++t) {
        if (rows[t] == 0) continue;
        const double2 *from = src[t];
        if (!on_dev) {
          e = hipMemcpyAsync(stage + off, src[t], sizeof(double2) * (size_t)rows[t] * npw, hipMemcpyHostToDevice, st);
          from = stage + off;
          off += (size_t)rows[t] * npw;
        }
        if (e == hipSuccess) e = launch_gather_rows(from, npw, ord, rows[t], dst[t], c->ld, st);
      }
      // the staging buffer is reused by the next entry
      if (e == hipSuccess && !on_dev) e = hipStreamSynchronize(st);
      if (e != hipSuccess) sst = fail(HP_ERR_HIP, "loading kpts[%d]: %s", i, hipGetErrorString(e));
    }
    if (stage) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(stage);
    }
    if (sst != HP_OK) return sst;
  }
  c->sk.sx = d_sx;
  c->sk.sy = d_sy;
  c->sk.sstart = d_ss;
  c->sk.slen = d_sl;
  c->sk.iz = d_iz;
  c->sk.xa = d_xa;
  c->sk.ent = d_ent;
  c->sk.max_pw256 = pw256;
  // row scales of the stacked projector table: D_i for beta rows, alpha for u rows
  std::vector<double> rs(c->n_proj);
  for (int b = 0; b < c->n_kb; ++b) rs[b] = gs->d_kb[b];
  for (int b = c->n_kb; b < c->n_beta; ++b) rs[b] = b < c->n_kb + 5 * c->n_hub ? 1.0 : -1.0;
  for (int v = 0; v < c->n_occ; ++v) rs[c->n_beta + v] = c->alpha;
  HPTRY(c->alloc(&c->d_rowscale, rs.size()));
  HPCHK(hipMemcpyAsync(c->d_rowscale, rs.data(), sizeof(double) * rs.size(), hipMemcpyHostToDevice, st));
  // energies of the mesh items
  const int nb = c->n_occ;
  const long nitems = (long)c->n_mesh * nb;
  std::vector<double> eps_items(nitems);
  for (int k = 0; k < c->n_mesh; ++k)
    for (int v = 0; v < nb; ++v) eps_items[(size_t)k * nb + v] = KP[k]->eps[v];
  HPTRY(c->alloc(&c->d_eps, nitems));
  HPCHK(hipMemcpyAsync(c->d_eps, eps_items.data(), sizeof(double) * nitems, hipMemcpyHostToDevice, st));
  // pairs
  HPTRY(c->alloc(&c->d_kp, c->n_mesh));
  HPTRY(c->alloc(&c->d_kself, c->n_kpts));
  std::vector<KPair> self(c->n_kpts);
  for (int i = 0; i < c->n_kpts; ++i) {
    self[i] = KPair{};
    self[i].ek = self[i].ej = i;
    self[i].spin = c->ent[i].spin;
    self[i].weight = c->ent[i].weight;
  }
  HPCHK(hipMemcpyAsync(c->d_kself, self.data(), sizeof(KPair) * self.size(), hipMemcpyHostToDevice, st));

  // work buffers
  const size_t vec = (size_t)nitems * c->ld;
  HPTRY(c->alloc(&c->B, vec));
  HPTRY(c->alloc(&c->X, vec));
  HPTRY(c->alloc(&c->R, vec));
  HPTRY(c->alloc(&c->P, vec));
  HPTRY(c->alloc(&c->AP, vec));
  HPTRY(c->alloc(&c->S1, (size_t)nitems * c->n3 * c->ns_pad));
  HPTRY(c->alloc(&c->S2, (size_t)nitems * c->n3 * c->ns_pad));
  const int mrow = std::max(c->n_proj, 5 * c->n_hub);
  HPTRY(c->alloc(&c->Cpart, (size_t)c->nsplit_cap * c->n_mesh * mrow * nb));
  HPTRY(c->alloc(&c->C, (size_t)c->n_mesh * mrow * nb));
  HPTRY(c->alloc(&c->Cphi, (size_t)c->n_mesh * 5 * c->n_hub * nb));
  HPTRY(c->alloc(&c->rz, nitems));
  HPTRY(c->alloc(&c->bn, nitems));
  HPTRY(c->alloc(&c->rn, nitems));
  HPTRY(c->alloc(&c->active, nitems));
  HPTRY(c->alloc(&c->bmap, (size_t)c->n_mesh * (nb + 1)));
  HPTRY(c->alloc(&c->count, kCntStep + kMaxChunk));
  HPTRY(c->alloc(&c->d_tol, 2));
  HPTRY(c->alloc(&c->d_stamps, 2 * kMaxStamps));
  {
    int dev = 0, khz = 0;
    HPCHK(hipGetDevice(&dev));
    HPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return fail(HP_ERR_HIP, "device reports no wall-clock rate");
    c->clock_khz = (double)khz;
  }
  // response density: the band loop of each (z plane, k) is split over drho_split workgroups
  // so that a launch has a few thousand of them
  c->drho_split = std::max(1, std::min(std::min(8, c->n_occ), (4096 + c->n3 * c->n_mesh - 1) / (c->n3 * c->n_mesh)));
  HPTRY(c->alloc(&c->part, (size_t)c->n_mesh * c->drho_split * c->nr));
  const size_t nv = (size_t)ns * c->nr;  // response fields: [nspin][nr]
  HPTRY(c->alloc(&c->drho, nv));
  HPTRY(c->alloc(&c->dvin, nv));
  HPTRY(c->alloc(&c->dvout, nv));
  HPTRY(c->alloc(&c->f, nv));
  HPTRY(c->alloc(&c->tmp, c->nr));
  HPTRY(c->alloc(&c->fprev, nv));
  HPTRY(c->alloc(&c->dvprev, nv));
  HPTRY(c->alloc(&c->hdf, (size_t)kNmixMax * nv));
  HPTRY(c->alloc(&c->hdv, (size_t)kNmixMax * nv));
  HPTRY(c->alloc(&c->dots_part, (size_t)256 * (2 * kNmixMax + 2)));
  HPTRY(c->alloc(&c->dots, 2 * kNmixMax + 2));
  HPTRY(c->alloc(&c->coef, 2 * kNmixMax + 2));
  HPTRY(c->alloc(&c->ptrs, 2 * kNmixMax + 2));
  HPTRY(c->alloc(&c->dn, (size_t)25 * c->n_hub));
  HPTRY(c->alloc(&c->d_q, 3));

  if (gs->projectors == HP_PROJ_ORTHO_ATOMIC) {
    std::vector<int> pw_offs(c->n_kpts);
    for (int i = 0; i < c->n_kpts; ++i) pw_offs[i] = h_ent[i].pw_off;
    HPTRY(ortho_atomic_projectors(c.get(), gs, KP, d_order, pw_offs));
  }
  if (gs->hub_pot) {
    // rows of the ground-state Hubbard potential from the final projectors of each entry:
    // chi_a = sum_m V_ma phi_m scaled by sqrt|lam_a| into the +1 (lam > 0) or -1 (lam < 0)
    // block of the stacked table, as one expansion on the matrix cores per entry with the
    // coefficients Cf[spin][5 s + m][r] (r = row in the 10 n_hub block); the Jacobi
    // diagonal below then gains sum_a lam_a |chi_a(G)|^2 through the row scales +-1
    const int nh = c->n_hub, nr10 = 10 * nh, nm = 5 * nh;
    std::vector<double2> cf((size_t)c->nspin * nm * nr10, make_double2(0.0, 0.0));
    for (int sp = 0; sp < c->nspin; ++sp)
      for (int sidx = 0; sidx < nh; ++sidx) {
        const int blk = sp * nh + sidx;
        for (int a = 0; a < 5; ++a) {
          const double lam = hub_lam[5 * blk + a];
          const double sc = std::sqrt(std::fabs(lam));
          const int r = (lam < 0.0 ? nm : 0) + 5 * sidx + a;
          for (int m = 0; m < 5; ++m) {
            const std::complex<double> z = sc * hub_vec[25 * blk + m * 5 + a];
            cf[((size_t)sp * nm + 5 * sidx + m) * nr10 + r] = make_double2(z.real(), z.imag());
          }
        }
      }
    double2 *d_cf = nullptr;
    HPTRY(dalloc(&d_cf, cf.size()));
    hipError_t e = hipMemcpyAsync(d_cf, cf.data(), sizeof(double2) * cf.size(), hipMemcpyHostToDevice, st);
    for (int i = 0; i < c->n_kpts && e == hipSuccess; ++i)
      e = launch_zexpand(c->d_kself + i, 0, 1, c->d_phi, c->phi_stride, 0, nm, d_cf + (size_t)spin_of[i] * nm * nr10,
                         (long)nm * nr10, 1.0, c->d_T + (size_t)i * c->t_stride + (size_t)c->n_kb * c->ld, c->ld, nr10,
                         c->d_npw, c->npw_max, nullptr, 1, st);
    const hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(d_cf);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return fail(HP_ERR_HIP, "ground-state Hubbard rows: %s", hipGetErrorString(e));
  }
  // Jacobi diagonal of every entry from the final stacked table and its row scales
  HPCHK(launch_diag(c->d_kself, c->sk.ent, c->n_kpts, c->d_T, c->t_stride, c->n_proj, c->d_rowscale, c->d_kin, d_vmean,
                    c->ld, c->d_diag, st));

  // A_k[m][v] = <phi_{m,k}|u_vk> for every entry (Eq. 13's ground-state factor)
  HPTRY(c->alloc(&c->d_A, (size_t)c->n_kpts * 5 * c->n_hub * nb));
  for (int i = 0; i < c->n_kpts; ++i) {
    HPTRY(proj(c.get(), c->d_kself + i, 0, 1, c->d_phi, c->phi_stride, 0, 5 * c->n_hub,
               c->d_T + (size_t)i * c->t_stride + (size_t)c->n_beta * c->ld, nb, nullptr, 1.0,
               c->d_A + (size_t)i * 5 * c->n_hub * nb));
  }
  // occupied states on the grid (permuted layout), every mesh k: psi[k*nb+v][z][plane]
  HPTRY(c->alloc(&c->d_psi, (size_t)nitems * c->nr));
  for (int k = 0; k < c->n_mesh; ++k)
    HPCHK(hipMemcpyAsync(c->X + (size_t)k * nb * c->ld, c->d_T + (size_t)k * c->t_stride + (size_t)c->n_beta * c->ld,
                         sizeof(double2) * (size_t)nb * c->ld, hipMemcpyDeviceToDevice, st));
  HPCHK(launch_stick_inv(c->sk, c->d_kself, 0, nb, (int)nitems, c->X, c->ld, c->S1, c->ns_pad, c->n3, c->az.tw,
                         c->max_chunk_pw, c->ns_max, nullptr, 0, st));
  HPCHK(launch_plane_to_real(c->pl, c->sk, c->d_kself, 0, nb, (int)nitems, c->S1, c->ns_pad, c->d_psi, st));
  HPTRY(sync(c.get()));
  if (c->degauss > 0.0) {
    // metals: projection weights, and for q = 0 the states at the Fermi level:
    // rho_F = 2 sum_k w sum_i (d_i / sigma) |u_i|^2 / Omega through the response-density
    // kernels (X = the kept bands scaled by d_i / (2 sigma), paired with themselves), and
    // n_F[s] = 2 sum_k w sum_i (d_i / sigma) <phi_m1|u_i><u_i|phi_m2>
    HPTRY(c->alloc(&c->d_beta, (size_t)c->n_mesh * nb * nb));
    HPTRY(c->alloc(&c->d_focc, (size_t)nitems));
    HPTRY(c->alloc(&c->d_rhoF, (size_t)c->nr));
    std::vector<double> cw(nitems);
    for (int k = 0; k < c->n_mesh; ++k)
      for (int v = 0; v < nb; ++v) cw[(size_t)k * nb + v] = c->occ_d[(size_t)k * nb + v] / (2.0 * c->degauss);
    HPCHK(hipMemcpyAsync(c->d_focc, cw.data(), sizeof(double) * cw.size(), hipMemcpyHostToDevice, st));
    HPCHK(launch_scale_rows((long)nitems * c->ld, c->ld, c->d_focc, c->X, st));
    HPCHK(launch_stick_inv(c->sk, c->d_kself, 1, nb, (int)nitems, c->X, c->ld, c->S1, c->ns_pad, c->n3, c->az.tw,
                           c->max_chunk_pw, c->ns_max, nullptr, 0, st));
    HPCHK(launch_plane_drho(c->pl, c->sk, c->d_kself, nb, c->n_mesh, c->S1, c->ns_pad, c->d_psi, c->part,
                            c->drho_split, st));
    HPCHK(launch_drho_reduce(c->d_kself, c->n_mesh, c->drho_split, c->part, c->nr, 1.0 / c->omega, c->occ, 1,
                             c->d_rhoF, st));
    const int M = 5 * c->n_hub;
    std::vector<double2> A((size_t)c->n_mesh * M * nb);
    HPCHK(hipMemcpyAsync(A.data(), c->d_A, sizeof(double2) * A.size(), hipMemcpyDeviceToHost, st));
    HPTRY(sync(c.get()));
    c->n_fermi.assign((size_t)25 * c->n_hub, 0.0);
    for (int k = 0; k < c->n_mesh; ++k)
      for (int v = 0; v < nb; ++v) {
        const double g = 2.0 * c->ent[k].weight * c->occ_d[(size_t)k * nb + v] / c->degauss;
        for (int s2 = 0; s2 < c->n_hub; ++s2)
          for (int m1 = 0; m1 < 5; ++m1)
            for (int m2 = 0; m2 < 5; ++m2) {
              const double2 a1 = A[((size_t)k * M + 5 * s2 + m1) * nb + v], a2 = A[((size_t)k * M + 5 * s2 + m2) * nb + v];
              c->n_fermi[(size_t)s2 * 25 + m1 * 5 + m2] +=
                  g * std::complex<double>(a1.x, a1.y) * std::conj(std::complex<double>(a2.x, a2.y));
            }
      }
  }
  *out = c.release();
  return HP_OK;
}

namespace {

hp_status run_scf(hp_ctx *c, int site, const double q[3], const hp_scf_params *p, double *dn0_out, double *dn_out,
                  hp_scf_stats *st) {
  Timer wall;
  const int nb = c->n_occ, nk = c->n_mesh, nitems = nk * nb;
  std::vector<KPair> pairs;
  HPTRY(upload_pairs(c, site, q, pairs));
  c->metal_q0 = false;
  if (c->degauss > 0.0) {
    HPTRY(upload_metal(c, pairs));
    c->metal_q0 = std::fabs(q[0] - std::round(q[0])) < 1e-12 && std::fabs(q[1] - std::round(q[1])) < 1e-12 &&
                  std::fabs(q[2] - std::round(q[2])) < 1e-12;
  }
  HPTRY(autotune(c, nk, p->precision == HP_MIXED));
  if (p->precision == HP_MIXED) HPTRY(setup32(c));
  HPCHK(hipMemcpyAsync(c->d_q, q, sizeof(double) * 3, hipMemcpyHostToDevice, c->stream));
  // response fields span every spin: [nspin][nr]
  const long nr = (long)c->nspin * c->nr;
  HPCHK(hipMemsetAsync(c->dvin, 0, sizeof(double2) * nr, c->stream));
  int nhist = 0, hist_head = 0;
  std::vector<std::complex<double>> gram((size_t)kNmixMax * kNmixMax);
  std::vector<double2> dn((size_t)25 * c->n_hub), dn0((size_t)25 * c->n_hub);
  std::vector<std::complex<double>> chi_prev;
  bool have_prev = false, converged = false;
  int it = 0, cg_total = 0, not_conv = 0;
  long happ = 0, happ32 = 0;
  double dchi = 0.0, vres = 1.0, max_rel = 0.0;
  double stage[8] = {0};
  for (it = 1; it <= p->niter_max; ++it) {
    // The first iteration gives chi0 and is solved to cg_tol; later iterations only need
    // the accuracy the response potential has reached (a fixed fraction of the last
    // mixing residual), never looser than 1e-3 nor tighter than cg_tol.
    const double tol_it = it == 1 ? p->cg_tol : std::max(p->cg_tol, std::min(1e-3, kAdaptiveTol * vres));
    // Mixed form, iterations solved no tighter than lowp_trust_tol: the RHS product and the
    // response density are accurate enough in FP32 (~1e-7 relative).
    const double trust_tol = p->lowp_trust_tol > 0.0 ? p->lowp_trust_tol : kFp32TrustTol;
    const bool lowp_it = p->precision == HP_MIXED && tol_it >= trust_tol;
    HPCHK(hipEventRecord(c->ev[0], c->stream));
    HPTRY(build_rhs(c, c->d_kp, nk, site, it > 1 ? c->dvin : nullptr, c->d_psi, lowp_it));
    HPCHK(hipEventRecord(c->ev[1], c->stream));
    int iters = 0, nc = 0, nref = 0;
    double mr = 0.0;
    if (p->precision == HP_MIXED) {
      HPTRY(cg_solve_mixed(c, c->d_kp, nk, c->d_eps, it > 1, tol_it, p->max_cg_iter, p->inner_tol, p->max_refine,
                           trust_tol,
                           &iters, &nc, &mr, &happ, &happ32, &nref));
    } else {
      HPTRY(cg_solve(c, c->d_kp, nk, c->d_eps, it > 1, tol_it, p->max_cg_iter, &iters, &nc, &mr, &happ));
    }
    HPCHK(hipEventRecord(c->ev[2], c->stream));
    cg_total += iters;
    not_conv = nc;
    max_rel = mr;
    // response density (spin x time reversal) and occupations (Eq. 13)
    if (lowp_it) {
      float2 *S1 = reinterpret_cast<float2 *>(c->S1);
      HPCHK(launch_to_f32((const double *)c->X, (float *)c->X32, 2L * nitems * c->ld, c->stream));
      HPCHK(timed(c, K_DRHO_STICKS, [&] {
        return launch_stick_inv32(c->sk, c->d_kp, 1, nb, nitems, c->X32, c->ld, S1, c->ns_pad, c->n3, c->az32.tw32,
                                  c->max_chunk_pw, c->ns_max, nullptr, stick_variant(c, 32, 0), c->stream);
      }));
      HPCHK(timed(c, K_PLANE_DRHO32, [&] {
        return launch_plane_drho32(c->pl32, c->sk, c->d_kp, nb, nk, S1, c->ns_pad, c->psi32, c->part, c->drho_split,
                                   c->stream);
      }));
    } else {
      HPCHK(timed(c, K_DRHO_STICKS, [&] {
        return launch_stick_inv(c->sk, c->d_kp, 1, nb, nitems, c->X, c->ld, c->S1, c->ns_pad, c->n3, c->az.tw,
                                c->max_chunk_pw, c->ns_max, nullptr, stick_variant(c, 64, 0), c->stream);
      }));
      HPCHK(timed(c, K_PLANE_DRHO, [&] {
        return launch_plane_drho(c->pl, c->sk, c->d_kp, nb, nk, c->S1, c->ns_pad, c->d_psi, c->part, c->drho_split,
                                 c->stream);
      }));
    }
    HPCHK(timed(c, K_DRHO_REDUCE, [&] {
      return launch_drho_reduce(c->d_kp, nk, c->drho_split, c->part, c->nr, 1.0 / c->omega, c->occ, c->nspin, c->drho,
                                c->stream);
    }));
    if (c->metal_q0) {  // Fermi-level shift: drho += shift * rho_F
      const double2 *xs[1] = {c->d_rhoF};
      const double2 cf[1] = {make_double2(c->fermi_shift.real(), c->fermi_shift.imag())};
      HPCHK(hipMemcpyAsync(c->ptrs, xs, sizeof(xs), hipMemcpyHostToDevice, c->stream));
      HPCHK(hipMemcpyAsync(c->coef, cf, sizeof(cf), hipMemcpyHostToDevice, c->stream));
      HPCHK(launch_zaxpy_list(c->nr, c->drho, 1, c->ptrs, c->coef, c->stream));
      HPTRY(sync(c));  // xs and cf live on this stack frame
    }
    HPCHK(hipEventRecord(c->ev[3], c->stream));
    HPCHK(timed(c, K_HXC, [&] {
      return launch_hxc(c->pl, c->az, c->d_bvec, q, c->drho, c->d_fxc, c->tmp, c->dvout, c->nspin, c->stream);
    }));
    HPCHK(hipEventRecord(c->ev[4], c->stream));
    HPTRY(proj(c, c->d_kp, 1, nk, c->d_phi, c->phi_stride, 0, 5 * c->n_hub, c->X, nb, nullptr, 1.0, c->Cphi));
    HPCHK(timed(c, K_DN, [&] {
      return launch_dn(c->d_kp, nk, c->n_hub, nb, c->d_A, c->Cphi, c->occ, c->dn, c->stream);
    }));
    HPCHK(hipMemcpyAsync(dn.data(), c->dn, sizeof(double2) * dn.size(), hipMemcpyDeviceToHost, c->stream));
    HPCHK(hipEventRecord(c->ev[5], c->stream));
    HPTRY(sync(c));
    if (c->metal_q0)  // Fermi-level shift of the occupations
      for (size_t i = 0; i < dn.size(); ++i) {
        const std::complex<double> t = c->fermi_shift * c->n_fermi[i];
        dn[i].x += t.real();
        dn[i].y += t.imag();
      }
    for (double2 z : dn)
      if (!std::isfinite(z.x) || !std::isfinite(z.y)) return fail(HP_ERR_NUMERIC, "non-finite response occupation");
    std::vector<std::complex<double>> chi(c->n_hub);
    for (int s = 0; s < c->n_hub; ++s) {
      std::complex<double> t = 0;
      for (int m = 0; m < 5; ++m) t += std::complex<double>(dn[s * 25 + m * 6].x, dn[s * 25 + m * 6].y);
      chi[s] = t;
    }
    if (it == 1) dn0 = dn;
    // mixing residual f = dV_out - dV_in
    HPCHK(timed(c, K_MIX, [&] {
      return launch_zsub(nr, c->dvout, c->dvin, c->f, c->stream);
    }));
    std::vector<std::complex<double>> nrm;
    {
      const double2 *v2[2] = {c->f, c->dvout};
      std::vector<std::complex<double>> a, b;
      HPTRY(zdots(c, 1, v2, c->f, nr, a));
      HPTRY(zdots(c, 1, v2 + 1, c->dvout, nr, b));
      const double fn = std::sqrt(std::max(0.0, a[0].real())), vn = std::sqrt(std::max(0.0, b[0].real()));
      vres = vn > 0 ? fn / vn : 0.0;
      if (!std::isfinite(vres)) return fail(HP_ERR_NUMERIC, "non-finite response potential");
    }
    if (have_prev) {
      dchi = 0.0;
      for (int s = 0; s < c->n_hub; ++s) dchi = std::max(dchi, std::abs(chi[s] - chi_prev[s]));
    }
    float ms[5];
    for (int s = 0; s < 5; ++s) (void)hipEventElapsedTime(&ms[s], c->ev[s], c->ev[s + 1]);
    for (int s = 0; s < 5; ++s) stage[s] += ms[s] * 1e-3;
    if (p->verbosity > 0)
      fprintf(stderr, "[hp] site %d q=(%.3f,%.3f,%.3f) it %d: dchi %.3e vres %.3e cg %d chi0/chi %.10f\n", site, q[0],
              q[1], q[2], it, have_prev ? dchi : NAN, vres, iters, chi[site].real());
    if (have_prev && dchi < p->conv_thr_chi && vres < p->conv_thr_v) {
      converged = true;
      break;
    }
    if (vres == 0.0) {  // no Hxc response at all
      converged = true;
      break;
    }
    chi_prev = chi;
    have_prev = true;
    if (it == p->niter_max) break;
    // modified Broyden (Anderson form) update of dV_in
    Timer tm;
    const int nmix = p->nmix;
    if (it > 1) {
      // new history pair from (f - f_prev, dv_in - dv_prev)
      double2 *df = c->hdf + (size_t)hist_head * nr;
      double2 *dvh = c->hdv + (size_t)hist_head * nr;
      HPCHK(timed(c, K_MIX, [&] {
        return launch_zsub(nr, c->f, c->fprev, df, c->stream);
      }));
      HPCHK(timed(c, K_MIX, [&] {
        return launch_zsub(nr, c->dvin, c->dvprev, dvh, c->stream);
      }));
      std::vector<std::complex<double>> d1;
      const double2 *v1[1] = {df};
      HPTRY(zdots(c, 1, v1, df, nr, d1));
      const double nd = std::sqrt(std::max(d1[0].real(), 1e-300));
      HPCHK(timed(c, K_MIX, [&] {
        return launch_zscale_copy(nr, df, 1.0 / nd, df, c->stream);
      }));
      HPCHK(timed(c, K_MIX, [&] {
        return launch_zscale_copy(nr, dvh, 1.0 / nd, dvh, c->stream);
      }));
      const int slot = hist_head;
      hist_head = (hist_head + 1) % nmix;
      nhist = std::min(nhist + 1, nmix);
      // Gram row of the new vector
      std::vector<const double2 *> vs;
      std::vector<int> slots;
      for (int h = 0; h < nhist; ++h) {
        const int sidx = ((hist_head - nhist + h) % nmix + nmix) % nmix;
        slots.push_back(sidx);
        vs.push_back(c->hdf + (size_t)sidx * nr);
      }
      std::vector<std::complex<double>> row;
      HPTRY(zdots(c, nhist, vs.data(), df, nr, row));  // <df_h | df_new>
      for (int h = 0; h < nhist; ++h) {
        gram[(size_t)slots[h] * kNmixMax + slot] = row[h];
        gram[(size_t)slot * kNmixMax + slots[h]] = std::conj(row[h]);
      }
    }
    HPCHK(hipMemcpyAsync(c->fprev, c->f, sizeof(double2) * nr, hipMemcpyDeviceToDevice, c->stream));
    HPCHK(hipMemcpyAsync(c->dvprev, c->dvin, sizeof(double2) * nr, hipMemcpyDeviceToDevice, c->stream));
    const double am = p->alpha_mix;
    std::vector<const double2 *> xs;
    std::vector<double2> cf;
    xs.push_back(c->f);
    cf.push_back(make_double2(am, 0.0));
    if (nhist > 0) {
      std::vector<int> slots;
      std::vector<const double2 *> vs;
      for (int h = 0; h < nhist; ++h) {
        const int sidx = ((hist_head - nhist + h) % nmix + nmix) % nmix;
        slots.push_back(sidx);
        vs.push_back(c->hdf + (size_t)sidx * nr);
      }
      std::vector<std::complex<double>> rhs;
      HPTRY(zdots(c, nhist, vs.data(), c->f, nr, rhs));  // <df_h | f>
      std::vector<std::complex<double>> G((size_t)nhist * nhist);
      for (int i = 0; i < nhist; ++i)
        for (int j = 0; j < nhist; ++j) G[(size_t)i * nhist + j] = gram[(size_t)slots[i] * kNmixMax + slots[j]];
      if (!csolve(nhist, G, rhs)) return fail(HP_ERR_NUMERIC, "singular mixing history");
      for (int h = 0; h < nhist; ++h) {
        const std::complex<double> g = rhs[h];
        xs.push_back(c->hdf + (size_t)slots[h] * nr);
        cf.push_back(make_double2(-am * g.real(), -am * g.imag()));
        xs.push_back(c->hdv + (size_t)slots[h] * nr);
        cf.push_back(make_double2(-g.real(), -g.imag()));
      }
    }
    HPCHK(hipMemcpyAsync(c->ptrs, xs.data(), sizeof(double2 *) * xs.size(), hipMemcpyHostToDevice, c->stream));
    HPCHK(hipMemcpyAsync(c->coef, cf.data(), sizeof(double2) * cf.size(), hipMemcpyHostToDevice, c->stream));
    HPCHK(timed(c, K_MIX, [&] {
      return launch_zaxpy_list(nr, c->dvin, (int)xs.size(), c->ptrs, c->coef, c->stream);
    }));
    HPTRY(sync(c));
    stage[4] += tm.s();
  }
  if (dn0_out)
    for (size_t i = 0; i < dn0.size(); ++i) {
      dn0_out[2 * i] = dn0[i].x;
      dn0_out[2 * i + 1] = dn0[i].y;
    }
  if (dn_out)
    for (size_t i = 0; i < dn.size(); ++i) {
      dn_out[2 * i] = dn[i].x;
      dn_out[2 * i + 1] = dn[i].y;
    }
  if (st) {
    st->scf_iters = std::min(it, p->niter_max);
    st->converged = converged ? 1 : 0;
    st->cg_iters = cg_total;
    st->h_applies_fp64 = happ;
    st->h_applies_lowp = happ32;
    st->wall_s = wall.s();
    st->chi_change = dchi;
    st->v_residual = vres;
    st->max_rel_resid = max_rel;
    for (int s = 0; s < 8; ++s) st->stage_s[s] = stage[s];
  }
  return (converged && not_conv == 0) ? HP_OK : HP_WARN_NOT_CONVERGED;
}

}  // namespace

extern "C" hp_status hp_sternheimer_scf(hp_ctx *c, int32_t pert_site, const double q_frac[3], const hp_scf_params *p,
                                        double *dn0_out, double *dn_out, hp_scf_stats *st) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (!q_frac || !dn0_out || !dn_out) return fail(HP_ERR_ARG, "NULL argument");
  HPTRY(check_params(p));
  apply_call_params(c, p);
  if (pert_site < 0 || pert_site >= c->n_hub) return fail(HP_ERR_ARG, "pert_site %d out of range", pert_site);
  if (st && st->struct_size != sizeof(hp_scf_stats)) return fail(HP_ERR_ARG, "hp_scf_stats.struct_size mismatch");
  return run_scf(c, pert_site, q_frac, p, dn0_out, dn_out, st);
}

extern "C" hp_status hp_response_matrix(hp_ctx *c, const int32_t nq[3], const hp_scf_params *p, double *chi0_out,
                                        double *chi_out, double *max_imag_out, hp_scf_stats *st) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (!nq || !chi0_out || !chi_out) return fail(HP_ERR_ARG, "NULL argument");
  HPTRY(check_params(p));
  apply_call_params(c, p);
  if (nq[0] < 1 || nq[1] < 1 || nq[2] < 1) return fail(HP_ERR_ARG, "nq must be >= 1");
  if (st && st->struct_size != sizeof(hp_scf_stats)) return fail(HP_ERR_ARG, "hp_scf_stats.struct_size mismatch");
  const int nh = c->n_hub;
  const int Nq = nq[0] * nq[1] * nq[2];
  std::vector<std::array<double, 3>> qs;
  for (int a = 0; a < nq[0]; ++a)
    for (int b = 0; b < nq[1]; ++b)
      for (int d = 0; d < nq[2]; ++d) qs.push_back({(double)a / nq[0], (double)b / nq[1], (double)d / nq[2]});
  // chi(q)[s][s'] for chi0 and chi
  std::vector<std::complex<double>> c0q((size_t)Nq * nh * nh), c1q((size_t)Nq * nh * nh);
  hp_status worst = HP_OK;
  hp_scf_stats acc{};
  acc.struct_size = sizeof(hp_scf_stats);
  std::vector<double> dn0(50 * nh), dn1(50 * nh);
  // sites to perturb: every site, or one per class of equal occupation trace
  std::vector<int> rep(nh);
  std::vector<double> moment(nh, 0.0);
  for (int s2 = 0; s2 < nh; ++s2) rep[s2] = s2;
  if (p->find_atpert == 1) {
    std::vector<double> trace;
    HPTRY(site_occupations(c, trace, moment));
    rep = site_classes(trace, p->docc_thr);
  }
  for (int iq = 0; iq < Nq; ++iq) {
    // time reversal: chi(-q) = conj chi(q); a q whose -q partner (modulo G) came earlier
    // in the mesh is not solved unless skip_equivalence_q is set
    int partner = -1;
    for (int j = 0; j < iq && !p->skip_equivalence_q && partner < 0; ++j) {
      bool same = true;
      for (int d = 0; d < 3; ++d) {
        const double t = qs[iq][d] + qs[j][d];
        same = same && std::fabs(t - std::round(t)) < 1e-9;
      }
      if (same) partner = j;
    }
    if (partner >= 0) {
      for (size_t e = 0; e < (size_t)nh * nh; ++e) {
        c0q[(size_t)iq * nh * nh + e] = std::conj(c0q[(size_t)partner * nh * nh + e]);
        c1q[(size_t)iq * nh * nh + e] = std::conj(c1q[(size_t)partner * nh * nh + e]);
      }
      continue;
    }
    for (int sp = 0; sp < nh; ++sp) {
      if (rep[sp] != sp) continue;
      hp_scf_stats one{};
      one.struct_size = sizeof(hp_scf_stats);
      hp_status s = run_scf(c, sp, qs[iq].data(), p, dn0.data(), dn1.data(), &one);
      if (s < 0) return s;
      if (s > worst) worst = s;
      acc.scf_iters += one.scf_iters;
      acc.cg_iters += one.cg_iters;
      acc.h_applies_fp64 += one.h_applies_fp64;
      acc.h_applies_lowp += one.h_applies_lowp;
      acc.wall_s += one.wall_s;
      acc.chi_change = std::max(acc.chi_change, one.chi_change);
      acc.v_residual = std::max(acc.v_residual, one.v_residual);
      acc.max_rel_resid = std::max(acc.max_rel_resid, one.max_rel_resid);
      for (int t = 0; t < 8; ++t) acc.stage_s[t] += one.stage_s[t];
      for (int s2 = 0; s2 < nh; ++s2) {
        std::complex<double> t0 = 0, t1 = 0;
        for (int m = 0; m < 5; ++m) {
          const int o = s2 * 25 + m * 6;
          t0 += std::complex<double>(dn0[2 * o], dn0[2 * o + 1]);
          t1 += std::complex<double>(dn1[2 * o], dn1[2 * o + 1]);
        }
        c0q[((size_t)iq * nh + s2) * nh + sp] = t0;
        c1q[((size_t)iq * nh + s2) * nh + sp] = t1;
      }
    }
  }
  // Eq. 12: chi_{(s,l),(s',l')} = (1/Nq) sum_q e^{i q.(R_l - R_l')} chi(q)_{s s'}
  const int n = nh * Nq;
  double mim = 0.0;
  std::vector<double> x0((size_t)n * n, 0.0), x1((size_t)n * n, 0.0);  // outputs, written at the end
  for (int l = 0; l < Nq; ++l)
    for (int lp = 0; lp < Nq; ++lp)
      for (int s = 0; s < nh; ++s)
        for (int sp = 0; sp < nh; ++sp) {
          if (rep[sp] != sp) continue;  // rebuilt below
          std::complex<double> a0 = 0, a1 = 0;
          for (int iq = 0; iq < Nq; ++iq) {
            const double dl[3] = {qs[l][0] * nq[0] - qs[lp][0] * nq[0], qs[l][1] * nq[1] - qs[lp][1] * nq[1],
                                  qs[l][2] * nq[2] - qs[lp][2] * nq[2]};
            const double ph = 2.0 * M_PI * (qs[iq][0] * dl[0] + qs[iq][1] * dl[1] + qs[iq][2] * dl[2]);
            const std::complex<double> e(std::cos(ph), std::sin(ph));
            a0 += e * c0q[((size_t)iq * nh + s) * nh + sp];
            a1 += e * c1q[((size_t)iq * nh + s) * nh + sp];
          }
          a0 /= (double)Nq;
          a1 /= (double)Nq;
          const int row = l * nh + s, col = lp * nh + sp;
          x0[(size_t)row * n + col] = a0.real();
          x1[(size_t)row * n + col] = a1.real();
          mim = std::max(mim, std::max(std::fabs(a0.imag()), std::fabs(a1.imag())));
        }
  if (p->find_atpert == 1) {
    // missing columns: copy chi[I2][J2] of a computed column with the classes of (I, J), the
    // same relative sign of the moments and the same distance within dist_thr
    const std::vector<double> D = supercell_distances(c->cell, nh, c->hub_tau.data(), nq);
    auto sgn = [&](int i) {
      const double m = moment[i % nh];
      return std::fabs(m) <= 1e-6 ? 0 : (m > 0 ? 1 : -1);
    };
    auto done = [&](int j) { return rep[j % nh] == j % nh; };
    std::vector<double> r0((size_t)n * n), r1((size_t)n * n);
    for (int J = 0; J < n; ++J) {
      if (done(J)) continue;
      for (int I = 0; I < n; ++I) {
        bool found = false;
        for (int J2 = 0; J2 < n && !found; ++J2) {
          if (!done(J2) || rep[J2 % nh] != rep[J % nh]) continue;
          for (int I2 = 0; I2 < n; ++I2)
            if (rep[I2 % nh] == rep[I % nh] && sgn(I2) * sgn(J2) == sgn(I) * sgn(J) &&
                std::fabs(D[(size_t)I2 * n + J2] - D[(size_t)I * n + J]) <= p->dist_thr) {
              r0[(size_t)I * n + J] = x0[(size_t)I2 * n + J2];
              r1[(size_t)I * n + J] = x1[(size_t)I2 * n + J2];
              found = true;
              break;
            }
        }
        if (!found)
          return fail(HP_ERR_ARG, "no computed element equivalent to chi[%d][%d] (dist_thr %g)", I, J, p->dist_thr);
      }
    }
    for (int J = 0; J < n; ++J)
      if (!done(J))
        for (int I = 0; I < n; ++I) {
          x0[(size_t)I * n + J] = r0[(size_t)I * n + J];
          x1[(size_t)I * n + J] = r1[(size_t)I * n + J];
        }
  }
  std::copy(x0.begin(), x0.end(), chi0_out);
  std::copy(x1.begin(), x1.end(), chi_out);
  if (max_imag_out) *max_imag_out = mim;
  if (st) *st = acc;
  return worst;
}

extern "C" hp_status hp_site_occupations(hp_ctx *c, double docc_thr, double *trace_out, double *moment_out,
                                         int32_t *class_out) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (!(docc_thr >= 0.0)) return fail(HP_ERR_ARG, "docc_thr must be >= 0");
  std::vector<double> trace, moment;
  HPTRY(site_occupations(c, trace, moment));
  const std::vector<int> rep = site_classes(trace, docc_thr);
  for (int s2 = 0; s2 < c->n_hub; ++s2) {
    if (trace_out) trace_out[s2] = trace[s2];
    if (moment_out) moment_out[s2] = moment[s2];
    if (class_out) class_out[s2] = rep[s2];
  }
  return HP_OK;
}

extern "C" hp_status hp_apply_h(hp_ctx *c, int32_t entry, int32_t n, const double *x, double *y) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (!x || !y) return fail(HP_ERR_ARG, "NULL argument");
  if (entry < 0 || entry >= c->n_kpts) return fail(HP_ERR_ARG, "entry %d out of range", entry);
  if (n < 1) return fail(HP_ERR_ARG, "n = %d out of range", n);
  entry = c->internal_of[entry];
  const HostEntry &E = c->ent[entry];
  const int cap = c->n_mesh * c->n_occ;  // vectors per batch (work-buffer capacity)
  std::vector<double2> h((size_t)cap * c->ld);
  for (int v0 = 0; v0 < n; v0 += cap) {
    const int nv = std::min(cap, n - v0);
    std::fill(h.begin(), h.end(), make_double2(0.0, 0.0));
    for (int v = 0; v < nv; ++v)
      for (int p = 0; p < E.npw; ++p) {
        const size_t q = (size_t)(v0 + v) * E.npw + E.order[p];
        h[(size_t)v * c->ld + p] = make_double2(x[2 * q], x[2 * q + 1]);
      }
    HPCHK(hipMemcpyAsync(c->P, h.data(), sizeof(double2) * (size_t)nv * c->ld, hipMemcpyHostToDevice, c->stream));
    HPTRY(apply_op(c, c->d_kself + entry, 0, 1, nv, c->P, c->AP, nullptr, c->n_beta));
    HPCHK(hipMemcpyAsync(h.data(), c->AP, sizeof(double2) * (size_t)nv * c->ld, hipMemcpyDeviceToHost, c->stream));
    HPTRY(sync(c));
    for (int v = 0; v < nv; ++v)
      for (int p = 0; p < E.npw; ++p) {
        const size_t q = (size_t)(v0 + v) * E.npw + E.order[p];
        y[2 * q] = h[(size_t)v * c->ld + p].x;
        y[2 * q + 1] = h[(size_t)v * c->ld + p].y;
      }
  }
  return HP_OK;
}

extern "C" hp_status hp_apply_h_lowp(hp_ctx *c, int32_t entry, int32_t n, int32_t lowp_gemm, const double *x,
                                     double *y) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (!x || !y) return fail(HP_ERR_ARG, "NULL argument");
  if (entry < 0 || entry >= c->n_kpts) return fail(HP_ERR_ARG, "entry %d out of range", entry);
  if (n < 1) return fail(HP_ERR_ARG, "n = %d out of range", n);
  if (lowp_gemm != HP_GEMM_FP32 && lowp_gemm != HP_GEMM_BF16 && lowp_gemm != HP_GEMM_BF16_PV32)
    return fail(HP_ERR_ARG, "unknown lowp_gemm %d", lowp_gemm);
  entry = c->internal_of[entry];
  const HostEntry &E = c->ent[entry];
  c->lowp_gemm = lowp_gemm;
  HPTRY(setup32(c));
  if (lowp_gemm != HP_GEMM_FP32) HPTRY(setup16(c));
  const int cap = c->n_mesh * c->n_occ;  // vectors per batch (work-buffer capacity)
  std::vector<float2> h((size_t)cap * c->ld);
  for (int v0 = 0; v0 < n; v0 += cap) {
    const int nv = std::min(cap, n - v0);
    std::fill(h.begin(), h.end(), make_float2(0.f, 0.f));
    for (int v = 0; v < nv; ++v)
      for (int p = 0; p < E.npw; ++p) {
        const size_t q = (size_t)(v0 + v) * E.npw + E.order[p];
        h[(size_t)v * c->ld + p] = make_float2((float)x[2 * q], (float)x[2 * q + 1]);
      }
    HPCHK(hipMemcpyAsync(c->P32, h.data(), sizeof(float2) * (size_t)nv * c->ld, hipMemcpyHostToDevice, c->stream));
    HPTRY(apply_op32(c, c->d_kself + entry, 1, nv, c->P32, c->AP32, nullptr, c->n_beta, nullptr));
    HPCHK(hipMemcpyAsync(h.data(), c->AP32, sizeof(float2) * (size_t)nv * c->ld, hipMemcpyDeviceToHost, c->stream));
    HPTRY(sync(c));
    for (int v = 0; v < nv; ++v)
      for (int p = 0; p < E.npw; ++p) {
        const size_t q = (size_t)(v0 + v) * E.npw + E.order[p];
        y[2 * q] = h[(size_t)v * c->ld + p].x;
        y[2 * q + 1] = h[(size_t)v * c->ld + p].y;
      }
  }
  return HP_OK;
}

// Bytes of workspace per vector of hp_apply_h_noalloc: X and H X in the stick order, the
// z-stick data before and after the plane round trip, the projection partial sums (at most
// nsplit_cap K slices) and the projections.
static size_t noalloc_bytes_per_vector(const hp_ctx *c) {
  return sizeof(double2) * (2 * (size_t)c->ld + 2 * (size_t)c->n3 * c->ns_pad +
                            (size_t)(c->nsplit_cap + 1) * std::max(c->n_beta, 1));
}

extern "C" hp_status hp_apply_h_noalloc(hp_ctx *c, int32_t entry, int32_t n, const double *x, double *y) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (!x || !y) return fail(HP_ERR_ARG, "NULL argument");
  if (entry < 0 || entry >= c->n_kpts) return fail(HP_ERR_ARG, "entry %d out of range", entry);
  const size_t per = noalloc_bytes_per_vector(c);
  const long nmax = (long)(HP_NOALLOC_SCRATCH_BYTES / per);
  if (n < 1 || n > nmax)
    return fail(HP_ERR_ARG, "n = %d out of range: the fixed %ld-byte workspace holds 1..%ld vectors of %zu bytes",
                n, (long)HP_NOALLOC_SCRATCH_BYTES, nmax, per);
  if (!c->scratch) return fail(HP_ERR_STATE, "no workspace for this context's device");
  for (const void *ptr : {(const void *)x, (const void *)y}) {  // host pointers would fault the kernels
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      return fail(HP_ERR_ARG, "x and y must be device memory");
    }
  }
  const int ie = c->internal_of[entry];
  const HostEntry &E = c->ent[ie];
  // workspace: X [n][ld] | Y [n][ld] | S1, S2 [n][n3][ns_pad] | Cpart [nsplit_cap][n_beta][n] | C [n_beta][n]
  double2 *X = reinterpret_cast<double2 *>(c->scratch);
  double2 *Y = X + (size_t)n * c->ld;
  OpWork w;
  w.S1 = Y + (size_t)n * c->ld;
  w.S2 = w.S1 + (size_t)n * c->n3 * c->ns_pad;
  w.Cpart = w.S2 + (size_t)n * c->n3 * c->ns_pad;
  w.C = w.Cpart + (size_t)c->nsplit_cap * std::max(c->n_beta, 1) * n;
  const int *ord = c->d_order + E.pw_off;
  HPCHK(launch_gather_rows(reinterpret_cast<const double2 *>(x), E.npw, ord, n, X, c->ld, c->stream));
  HPTRY(apply_op(c, c->d_kself + ie, 0, 1, n, X, Y, nullptr, c->n_beta, nullptr, &w));
  HPCHK(launch_scatter_rows(Y, c->ld, E.npw, ord, n, reinterpret_cast<double2 *>(y), c->stream));
  return HP_OK;
}

extern "C" hp_status hp_solve_first_order(hp_ctx *c, int32_t pert_site, const double q_frac[3], int32_t mesh_k,
                                          const double *dv, const hp_scf_params *p, double *du_out) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (!q_frac || !du_out) return fail(HP_ERR_ARG, "NULL argument");
  HPTRY(check_params(p));
  apply_call_params(c, p);
  if (pert_site < 0 || pert_site >= c->n_hub) return fail(HP_ERR_ARG, "pert_site out of range");
  if (mesh_k < 0 || mesh_k >= c->n_mesh) return fail(HP_ERR_ARG, "mesh_k out of range");
  std::vector<KPair> pairs;
  HPTRY(upload_pairs(c, pert_site, q_frac, pairs));
  const KPair P = pairs[mesh_k];
  HPCHK(hipMemcpyAsync(c->d_kp, &P, sizeof(KPair), hipMemcpyHostToDevice, c->stream));
  c->metal_q0 = false;  // a single k: no Fermi-level shift here
  if (c->degauss > 0.0) HPTRY(upload_metal(c, std::vector<KPair>{P}));
  HPTRY(autotune(c, 1, p->precision == HP_MIXED));
  const int nb = c->n_occ;
  const double2 *psi = c->d_psi + (size_t)mesh_k * nb * c->nr;
  const double *eps = c->d_eps + (size_t)mesh_k * nb;
  if (dv) {
    for (int sp = 0; sp < c->nspin; ++sp) {
      HPCHK(hipMemcpyAsync(c->tmp, dv + 2 * (size_t)sp * c->nr, sizeof(double2) * c->nr, hipMemcpyHostToDevice,
                           c->stream));
      HPCHK(launch_permute_complex(c->pl, c->d_px, c->d_py, c->tmp, c->dvin + (size_t)sp * c->nr, 0, c->stream));
    }
  }
  // A for this k: build_rhs indexes d_A by pair index; use a shifted view
  hp_status s = HP_OK;
  {
    // temporarily point the perturbation factor at entry mesh_k
    double2 *saveA = c->d_A;
    c->d_A = c->d_A + (size_t)mesh_k * 5 * c->n_hub * nb;
    s = build_rhs(c, c->d_kp, 1, pert_site, dv ? c->dvin : nullptr, psi);
    c->d_A = saveA;
    if (s < 0) return s;
  }
  int iters = 0, nc = 0, nref = 0;
  double mr = 0.0;
  long happ = 0, happ32 = 0;
  if (p->precision == HP_MIXED) {
    HPTRY(cg_solve_mixed(c, c->d_kp, 1, eps, 0, p->cg_tol, p->max_cg_iter, p->inner_tol, p->max_refine,
                         p->lowp_trust_tol > 0.0 ? p->lowp_trust_tol : kFp32TrustTol, &iters, &nc,
                         &mr, &happ, &happ32, &nref));
  } else {
    HPTRY(cg_solve(c, c->d_kp, 1, eps, 0, p->cg_tol, p->max_cg_iter, &iters, &nc, &mr, &happ));
  }
  const HostEntry &E = c->ent[P.ej];
  std::vector<double2> h((size_t)nb * c->ld);
  HPCHK(hipMemcpyAsync(h.data(), c->X, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HPTRY(sync(c));
  for (int v = 0; v < nb; ++v)
    for (int p2 = 0; p2 < E.npw; ++p2) {
      const int q = E.order[p2];
      du_out[2 * ((size_t)v * E.npw + q)] = h[(size_t)v * c->ld + p2].x;
      du_out[2 * ((size_t)v * E.npw + q) + 1] = h[(size_t)v * c->ld + p2].y;
    }
  return nc == 0 ? HP_OK : HP_WARN_NOT_CONVERGED;
}

extern "C" hp_status hp_xc_kernel(int32_t nspin, int64_t n, const double *rho, double *fxc_out) {
  if (!rho || !fxc_out) return fail(HP_ERR_ARG, "NULL argument");
  if (nspin != 1 && nspin != 2) return fail(HP_ERR_ARG, "nspin must be 1 or 2");
  if (n < 1) return fail(HP_ERR_ARG, "n must be >= 1");
  const size_t nin = (size_t)nspin * n, nout = (size_t)(nspin == 2 ? 3 : 1) * n;
  double *d_in = nullptr, *d_out = nullptr;
  HPTRY(dalloc(&d_in, nin));
  hp_status s = dalloc(&d_out, nout);
  if (s == HP_OK) {
    hipError_t e = hipMemcpy(d_in, rho, sizeof(double) * nin, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = nspin == 2 ? launch_fxc_spin(d_in, d_in + n, d_out, n, nullptr) : launch_fxc(d_in, d_out, n, nullptr);
    if (e == hipSuccess) e = hipMemcpy(fxc_out, d_out, sizeof(double) * nout, hipMemcpyDeviceToHost);
    if (e != hipSuccess) s = fail(HP_ERR_HIP, "hp_xc_kernel: %s", hipGetErrorString(e));
  }
  (void)hipFree(d_in);
  if (d_out) (void)hipFree(d_out);
  return s;
}

extern "C" hp_status hp_profile_start(hp_ctx *c) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  HPTRY(sync(c));
  c->prof_on = true;
  for (int i = 0; i < K_COUNT; ++i) {
    c->prof_calls[i] = 0;
    c->prof_ms[i] = 0.0;
  }
  return HP_OK;
}

extern "C" hp_status hp_profile_stop(hp_ctx *c, hp_kernel_time *out, int32_t max, int32_t *n_out) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  HPTRY(sync(c));
  c->prof_on = false;
  int n = 0;
  for (int i = 0; i < K_COUNT; ++i) {
    if (out && n < max) {
      out[n].name = kKernelNames[i];
      out[n].calls = c->prof_calls[i];
      out[n].total_ms = c->prof_ms[i];
    }
    ++n;
  }
  if (n_out) *n_out = std::min(n, max);
  return HP_OK;
}

extern "C" hp_status hp_tuning_report(hp_ctx *c, char *buf, int32_t len) {
  if (!c || !buf || len < 1) return fail(HP_ERR_ARG, "NULL argument or len < 1");
  static const char *const kTile[4] = {"32x32", "64x32", "32x64", "64x64"};
  std::string o = "{\"gemm\": [";
  char line[512];
  for (size_t i = 0; i < c->gemm_tuned.size(); ++i) {
    const auto &g = c->gemm_tuned[i];
    snprintf(line, sizeof line,
             "%s{\"prec\": %d, \"rows\": %d, \"batch\": %d, \"proj_tile\": \"%s\", \"nsplit\": %d, "
             "\"expand_bands\": %d, \"proj_ms\": %.4f, \"proj_default_ms\": %.4f, \"expand_ms\": %.4f, "
             "\"expand_default_ms\": %.4f}",
             i ? ", " : "", g.prec, g.M, g.nk, kTile[g.tile & 3], g.ns, 32 * g.bv, g.proj_ms, g.proj_default_ms,
             g.expand_ms, g.expand_default_ms);
    o += line;
  }
  o += "], \"plane\": [";
  bool first = true;
  for (int slot = 0; slot < 2; ++slot) {
    if (!c->plane_tuned[slot]) continue;
    snprintf(line, sizeof line, "%s{\"prec\": %d, \"variant\": %d, \"ms\": [", first ? "" : ", ",
             slot ? 32 : 64, c->plane_var[slot]);
    o += line;
    for (int v = 0; v < c->plane_nvar[slot]; ++v) {
      snprintf(line, sizeof line, "%s%.4f", v ? ", " : "", c->plane_ms[slot][v]);
      o += line;
    }
    o += "]}";
    first = false;
  }
  o += "], \"sticks\": [";
  first = true;
  for (int slot = 0; slot < 2; ++slot) {
    if (!c->stick_tuned[slot]) continue;
    snprintf(line, sizeof line,
             "%s{\"prec\": %d, \"inverse_variant\": %d, \"inverse_ms\": [%.4f, %.4f, %.4f], "
             "\"forward_variant\": %d, \"forward_ms\": [%.4f, %.4f, %.4f]}",
             first ? "" : ", ", slot ? 32 : 64, c->stick_var[slot][0], c->stick_ms[slot][0][0], c->stick_ms[slot][0][1],
             c->stick_ms[slot][0][2], c->stick_var[slot][1], c->stick_ms[slot][1][0], c->stick_ms[slot][1][1],
             c->stick_ms[slot][1][2]);
    o += line;
    first = false;
  }
  o += "]}";
  if ((int32_t)o.size() + 1 > len) return fail(HP_ERR_ARG, "buffer too small (%d bytes needed)", (int)o.size() + 1);
  memcpy(buf, o.c_str(), o.size() + 1);
  return HP_OK;
}

// Captured graphs bake in launch shapes: drop them when a shape is pinned.
static void drop_graphs(hp_ctx *c) {
  (void)hipStreamSynchronize(c->stream);
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

extern "C" hp_status hp_set_gemm_shape(hp_ctx *c, int32_t prec, int32_t rows, int32_t batch, int32_t tile,
                                       int32_t nsplit, int32_t expand_bands) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (prec != 64 && prec != 32 && prec != 16) return fail(HP_ERR_ARG, "prec must be 64, 32 or 16");
  if (rows < 1 || batch < 1 || batch > c->n_mesh) return fail(HP_ERR_ARG, "bad rows/batch");
  if (tile < 0 || tile > 3) return fail(HP_ERR_ARG, "tile must be in 0..3");
  if (nsplit < 1 || nsplit > c->nsplit_cap) return fail(HP_ERR_ARG, "nsplit must be in 1..%d", c->nsplit_cap);
  if (expand_bands != 32 && expand_bands != 64 && expand_bands != 128)
    return fail(HP_ERR_ARG, "expand_bands must be 32, 64 or 128");
  hp_ctx::GemmChoice g{prec, rows, batch, tile, nsplit, expand_bands / 32, 0.f, 0.f, 0.f, 0.f};
  drop_graphs(c);
  for (auto &e : c->gemm_tuned)
    if (e.prec == prec && e.M == rows && e.nk == batch) {
      e = g;
      return HP_OK;
    }
  c->gemm_tuned.push_back(g);
  return HP_OK;
}

extern "C" hp_status hp_set_plane_variant(hp_ctx *c, int32_t prec, int32_t variant) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (prec != 64 && prec != 32) return fail(HP_ERR_ARG, "prec must be 64 or 32");
  const int slot = prec == 32 ? 1 : 0;
  if (!plane_vloc_variant_ok(c->pl, prec == 32 ? (int)sizeof(float2) : (int)sizeof(double2), variant))
    return fail(HP_ERR_ARG, "plane variant %d is not available for this grid", variant);
  const int nv = kPlaneVariants;
  c->plane_var[slot] = variant;
  c->plane_nvar[slot] = nv;
  c->plane_tuned[slot] = true;
  drop_graphs(c);
  return HP_OK;
}

extern "C" hp_status hp_set_stick_variant(hp_ctx *c, int32_t prec, int32_t inverse_variant, int32_t forward_variant) {
  if (!c) return fail(HP_ERR_ARG, "context is NULL");
  if (prec != 64 && prec != 32) return fail(HP_ERR_ARG, "prec must be 64 or 32");
  const int nv = stick_variants(c);
  if (inverse_variant < 0 || inverse_variant >= nv || forward_variant < 0 || forward_variant >= nv)
    return fail(HP_ERR_ARG, "variants must be in 0..%d for this grid", nv - 1);
  const int slot = prec == 32 ? 1 : 0;
  c->stick_var[slot][0] = inverse_variant;
  c->stick_var[slot][1] = forward_variant;
  c->stick_tuned[slot] = true;
  drop_graphs(c);
  return HP_OK;
}
