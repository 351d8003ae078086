// libtnrg: kernels and C ABI of the MPS robust-GRAPE hot path for gfx950.
// The ABI is declared and documented in include/tnrg.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>

#include "tnrg.h"
#include "tnrg_common.hpp"

using namespace tnrg;

// ============================================================================
// Gate table: for slice l and site j, the half-slice rotation
//   R = exp(-i (dt/2) (ux X + uy Y)/2) = cos(a r) I - i sin(a r)/r (ux X + uy Y),
// a = dt/4, r = |(ux, uy)|, and its derivatives
//   dR/dux = -a ux f I - i (g ux n + f X),  dR/duy = -a uy f I - i (g uy n + f Y)
// with n = ux X + uy Y, f = sin(a r)/r, g = f'(r)/r (Sec. III, Eq. 8 drive).
// Near r = 0, f and g are evaluated from their Taylor series.
__device__ __forceinline__ void half_rotation_f_g(double a, double r, double* f, double* g) {
  const double x = a * r;
  if (x < 0.1) {
    const double x2 = x * x;
    // sin(x)/x = 1 - x^2/6 + x^4/120 - x^6/5040 + x^8/362880 - x^10/39916800
    *f = a * (1.0 + x2 * (-1.0 / 6.0 + x2 * (1.0 / 120.0 + x2 * (-1.0 / 5040.0 +
                                                                 x2 * (1.0 / 362880.0 - x2 / 39916800.0)))));
    // (x cos x - sin x)/x^3 = -1/3 + x^2/30 - x^4/840 + x^6/45360 - x^8/3991680
    *g = a * a * a * (-1.0 / 3.0 + x2 * (1.0 / 30.0 + x2 * (-1.0 / 840.0 +
                                                            x2 * (1.0 / 45360.0 - x2 / 3991680.0))));
  } else {
    double sx, cx;
    sincos(x, &sx, &cx);
    *f = sx / r;
    *g = (x * cx - sx) / (r * r * r);
  }
}

__global__ void k_gates(int M, int N, double dt, int order, const double* __restrict__ ux,
                        const double* __restrict__ uy, c2* __restrict__ gates) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const double x = ux[idx], y = uy[idx];
  if (order == 1) {
    // first-order split: the drive factor of the slice is G = Xr Yr with
    // Xr = exp(-i dt x X/2), Yr = exp(-i dt y Y/2); stored as G, dG/dux =
    // (-i dt/2 X) G and dG/duy = Xr (-i dt/2 Y) Yr
    double sx, cx, sy, cy;
    sincos(0.5 * dt * x, &sx, &cx);
    sincos(0.5 * dt * y, &sy, &cy);
    M22 Xr, Yr, Xh, Yh;
    Xr.m[0] = cmk(cx, 0.0); Xr.m[1] = cmk(0.0, -sx); Xr.m[2] = cmk(0.0, -sx); Xr.m[3] = cmk(cx, 0.0);
    Yr.m[0] = cmk(cy, 0.0); Yr.m[1] = cmk(-sy, 0.0); Yr.m[2] = cmk(sy, 0.0); Yr.m[3] = cmk(cy, 0.0);
    const double h = -0.5 * dt;
    // -i dt/2 X and -i dt/2 Y
    Xh.m[0] = cmk(0.0, 0.0); Xh.m[1] = cmk(0.0, h); Xh.m[2] = cmk(0.0, h); Xh.m[3] = cmk(0.0, 0.0);
    Yh.m[0] = cmk(0.0, 0.0); Yh.m[1] = cmk(h, 0.0); Yh.m[2] = cmk(-h, 0.0); Yh.m[3] = cmk(0.0, 0.0);
    const M22 G = m22_mul(Xr, Yr);
    const M22 dGx = m22_mul(Xh, G);
    const M22 dGy = m22_mul(m22_mul(Xr, Yh), Yr);
    c2* o = gates + (size_t)idx * 12;
    for (int q = 0; q < 4; ++q) {
      o[q] = G.m[q];
      o[4 + q] = dGx.m[q];
      o[8 + q] = dGy.m[q];
    }
    return;
  }
  const double a = 0.25 * dt;
  const double r = sqrt(x * x + y * y);
  double f, g;
  half_rotation_f_g(a, r, &f, &g);
  const double c = cos(a * r);
  c2* o = gates + (size_t)idx * 12;
  // R = c I - i f (x X + y Y):  X = [[0,1],[1,0]], Y = [[0,-i],[i,0]]
  // x X + y Y = [[0, x - i y], [x + i y, 0]]
  // -i f (x - i y) = -f y - i f x ;  -i f (x + i y) = f y - i f x
  o[0] = cmk(c, 0.0);
  o[1] = cmk(-f * y, -f * x);
  o[2] = cmk(f * y, -f * x);
  o[3] = cmk(c, 0.0);
  // dR/dux = -a x f I - i (g x (x X + y Y) + f X)
  {
    const double gx = g * x;
    // off-diagonal of g x n + f X:  [0,1]: gx (x - i y) + f ; [1,0]: gx (x + i y) + f
    const c2 u01 = cmk(gx * x + f, -gx * y);
    const c2 u10 = cmk(gx * x + f, gx * y);
    o[4] = cmk(-a * x * f, 0.0);
    o[5] = cmk(u01.y, -u01.x);  // -i * u01
    o[6] = cmk(u10.y, -u10.x);
    o[7] = cmk(-a * x * f, 0.0);
  }
  // dR/duy = -a y f I - i (g y (x X + y Y) + f Y);  f Y = [[0, -i f], [i f, 0]]
  {
    const double gy = g * y;
    const c2 u01 = cmk(gy * x, -gy * y - f);
    const c2 u10 = cmk(gy * x, gy * y + f);
    o[8] = cmk(-a * y * f, 0.0);
    o[9] = cmk(u01.y, -u01.x);
    o[10] = cmk(u10.y, -u10.x);
    o[11] = cmk(-a * y * f, 0.0);
  }
}


// ============================================================================
// Kernel arguments (shared by both memory-space variants).
// Persistent fidelity+gradient kernel: one workgroup per trajectory (k, r).
struct GrapeArgs {
  ModelDev md;
  const double* ux;
  const double* uy;
  const double* uzz;
  const double* J;
  int K, R;
  const c2* in_data;
  const int* in_dims;
  int in_dcap;
  long long in_stride;
  const c2* tg_data;
  const int* tg_dims;
  int tg_dcap;
  long long tg_stride;
  int dcap, cs, nck, nslots, nctrl;
  const c2* gates;
  int* flags;
  long long* stats;
  char* traj_base;
  size_t traj_bytes, slot_bytes, dims_off, off_x0, off_env, off_O, off_g;
  size_t off_env2;  // mid-sweep u^zz insertions: right envs (N+1) cap^2 + 2 cap^2
  size_t off_big;  // working buffers of the global-scratch variant (capacities above 32)
  c2* overlaps;
  c2* traj_dO;
  int mode;                // kModeForward | kModeBackward
  unsigned long long tag;  // fingerprint of the call's arguments
  int jx_elems;            // global-scratch build: LDS for the Jacobi matrix (complex)
};


constexpr int kModeForward = 1, kModeBackward = 2;


// mps_evolve kernel: one workgroup per trajectory, slices in place.
struct EvolveArgs {
  ModelDev md;
  const double* uzz;
  const double* J;
  const c2* gates;
  c2* data;
  int* dims;
  int dcap;
  long long stride;
  int l_begin, l_end, adjoint;
  c2* x0;
  c2* big;  // working buffers of the global-scratch variant, big_stride per trajectory
  size_t big_stride;
  int* flags;
  long long* stats;
  int jx_elems;  // global-scratch build: LDS for the Jacobi matrix (complex)
};


// mps_overlap kernel: out[t] = <bra_{t % nb} | ket_t>.
struct OverlapArgs {
  ModelDev md;
  const c2* bra;
  const int* bdims;
  int bdcap;
  long long bstride;
  int nb;
  const c2* ket;
  const int* kdims;
  int kdcap;
  long long kstride;
  int cap;
  c2* out;
  int* flags;
  c2* big;
  size_t big_stride;
};


// Deterministic ensemble reduction: F = mean |O_t|^2, grad = mean of the
// per-trajectory 2 Re(conj O dO) (Sec. II, Eq. 7), summed in trajectory order.
__global__ void k_reduce(int n_traj, int nctrl, int MN, int MN1, const char* traj_base,
                         size_t traj_bytes, size_t off_O, size_t off_g, double* F, double* gux,
                         double* guy, double* guzz) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const double inv = 1.0 / (double)n_traj;
  if (c < nctrl) {
    double s = 0.0;
    for (int t = 0; t < n_traj; ++t)
      s += reinterpret_cast<const double*>(traj_base + (size_t)t * traj_bytes + off_g)[c];
    s *= inv;
    if (c < MN)
      gux[c] = s;
    else if (c < 2 * MN)
      guy[c - MN] = s;
    else
      guzz[c - 2 * MN] = s;
  }
  if (c == 0 && F) {
    double s = 0.0;
    for (int t = 0; t < n_traj; ++t) {
      const c2 o = *reinterpret_cast<const c2*>(traj_base + (size_t)t * traj_bytes + off_O);
      s += cabs2(o);
    }
    F[0] = s * inv;
  }
}


// The two variants of the persistent kernels.
#define TNRG_NS lds
#define TNRG_AS __attribute__((address_space(3)))
#define TNRG_BIG 0
#include "tnrg_device.hpp"
#include "tnrg_kernels.inc"
#undef TNRG_NS
#undef TNRG_AS
#undef TNRG_BIG
#define TNRG_NS big
#define TNRG_AS
#define TNRG_BIG 1
#include "tnrg_device.hpp"
#include "tnrg_kernels.inc"
#undef TNRG_NS
#undef TNRG_AS
#undef TNRG_BIG

// Working buffers of one workgroup for capacity cap (LDS in the first
// variant, global scratch in the second).
static size_t dyn_lds_bytes(int cap) {
  size_t P2 = 4;
  while (P2 < (size_t)2 * cap) P2 <<= 1;
  return (P2 * P2 + P2 * (P2 + 1)) * sizeof(c2) + P2 * sizeof(double) + P2 * sizeof(int);
}


// ============================================================================
// Host side: validation, workspace layout, launches.
namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(TNRG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

// Shared with the serving runtime (tnrg_server.cpp); not exported.
__attribute__((visibility("hidden"))) int tnrg_set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_model(const tnrg_model* md, ModelDev* out) {
  if (!md) return fail(TNRG_EINVAL, "model is NULL");
  if (md->n < 2 || md->n > kMaxSites) return fail(TNRG_EINVAL, "n = %d outside [2, %d]", md->n, kMaxSites);
  if (md->m < 1) return fail(TNRG_EINVAL, "m = %d < 1", md->m);
  if (!(md->dt > 0.0) || !isfinite(md->dt)) return fail(TNRG_EINVAL, "dt must be finite and > 0");
  if (md->chi < 1) return fail(TNRG_EINVAL, "chi = %d < 1", md->chi);
  if (!(md->trunc_eps >= 0.0) || !isfinite(md->trunc_eps))
    return fail(TNRG_EINVAL, "trunc_eps must be finite and >= 0");
  if (md->max_sweeps < 0) return fail(TNRG_EINVAL, "max_sweeps < 0");
  if (md->split_order != 0 && md->split_order != 1 && md->split_order != 2)
    return fail(TNRG_EINVAL, "split_order = %d must be 0, 1 or 2", md->split_order);
  if (md->xt_model != 0 && md->xt_model != 1)
    return fail(TNRG_EINVAL, "xt_model = %d must be 0 or 1", md->xt_model);
  if (!md->zz_mask || !md->xt_mask) return fail(TNRG_EINVAL, "bond masks must be host arrays");
  ModelDev d;
  memset(&d, 0, sizeof d);
  d.N = md->n;
  d.M = md->m;
  d.dt = md->dt;
  d.chi = md->chi;
  d.eps = md->trunc_eps;
  d.renorm = md->renormalize ? 1 : 0;
  d.max_sweeps = md->max_sweeps > 0 ? md->max_sweeps : 40;
  d.profile = md->profile ? 1 : 0;
  d.order = md->split_order == 1 ? 1 : 2;
  d.heis = md->xt_model == 1 ? 1 : 0;
  d.zz_lo = md->n - 1;
  d.zz_hi = -1;
  for (int b = 0; b < md->n - 1; ++b) {
    if (md->zz_mask[b]) {
      d.zzm[b >> 6] |= 1ull << (b & 63);
      d.zz_lo = std::min(d.zz_lo, b);
      d.zz_hi = std::max(d.zz_hi, b);
    }
    if (md->xt_mask[b]) d.xtm[b >> 6] |= 1ull << (b & 63);
  }
  d.hgrad = d.heis && d.zz_hi >= 0;
  *out = d;
  return TNRG_OK;
}

int check_batch(const tnrg_mps_batch* b, int N, const char* name) {
  if (!b) return fail(TNRG_EINVAL, "%s is NULL", name);
  if (b->n_sites != N) return fail(TNRG_EINVAL, "%s has %d sites, model has %d", name, b->n_sites, N);
  if (b->n_traj < 1) return fail(TNRG_EINVAL, "%s has no trajectories", name);
  if (b->dcap < 1) return fail(TNRG_EINVAL, "%s dcap < 1", name);
  if (!b->bond_dim || !b->data) return fail(TNRG_EINVAL, "%s has NULL device pointers", name);
  return TNRG_OK;
}

// Threads per workgroup for a capacity bucket: enough lanes for every
// column pair of a (2 cap) x (2 cap) Jacobi round with >= 2 lanes per pair.
// The launch plan (set by the autotuner through tnrg_plan_set_threads)
// overrides this per capacity.
std::atomic<int> g_plan_threads[kMaxSites + 1];

// Fewest threads for the LDS variant at capacity cap: every Jacobi round
// processes up to cap column pairs at once with at least pow2(2 cap) / 8 lanes
// each (8 rows per lane).  The global-scratch variant loops over the pairs of
// a round and runs with any workgroup size.
int min_threads_lds(int cap) {
  int p2 = 1;
  while (p2 < 2 * cap) p2 <<= 1;
  const int need = (p2 / 8 > 1 ? p2 / 8 : 1) * cap;
  int nt = 64;
  while (nt < need) nt *= 2;
  return nt;
}

bool use_lds(int cap);

int threads_for_cap(int cap) {
  const int lo = use_lds(cap) ? min_threads_lds(cap) : 64;
  if (cap >= 0 && cap <= kMaxSites) {
    const int t = g_plan_threads[cap].load(std::memory_order_relaxed);
    if (t >= lo) return t;
  }
  return use_lds(cap) ? lo : 256;
}

// Largest dynamic LDS a workgroup may use on gfx950.
constexpr size_t kMaxDynLds = 160 * 1024 - sizeof(lds::Shared) - 512;
// The global-scratch build can run the Jacobi of a bond update on an LDS
// copy of its matrix (when rank x (pow2(len) + 1) + 2 pow2(len) complex fit):
// LDS round trips instead of L2 ones, at the price of one workgroup per CU.
// Measured at dcap 64 (N = 50, Heisenberg crosstalk): 21 % faster with one
// trajectory per CU, 31 % with two (the co-resident workgroups of the
// global-scratch Jacobi do not overlap), so it is the default at any count.
// Mode -1 (default) and 1: on; 0: off.
constexpr size_t kBigJacLds = (160 * 1024 - sizeof(big::Shared) - 512) / 16 * 16;
std::atomic<int> g_jacobi_lds{-1};
int jacobi_lds_elems() {
  return g_jacobi_lds.load(std::memory_order_relaxed) == 0 ? 0 : (int)(kBigJacLds / sizeof(c2));
}
// Capacities up to kMaxLdsCap keep the working buffers in LDS; larger ones
// (up to kMaxCap: a 2 cap x 2 cap bond problem of at most 256 columns for the
// wave-level pivot search and sort) in per-trajectory global scratch.
constexpr int kMaxLdsCap = 32;
constexpr int kMaxCap = 128;
bool use_lds(int cap) { return cap <= kMaxLdsCap && dyn_lds_bytes(cap) <= kMaxDynLds; }
size_t big_bytes(int cap) { return use_lds(cap) ? 0 : align256(dyn_lds_bytes(cap)); }

struct GrapeLayout {
  int cs, nck, nslots, nctrl, dcap;
  size_t slot_bytes, dims_off, off_x0, off_env, off_env2, off_O, off_g, off_big, traj_bytes;
  size_t off_flags, off_stats, off_gates, off_traj, total;
};

// Heisenberg crosstalk with some u^zz control: the adjoint takes the u^zz
// derivative inside its sweeps (more workspace: one MPS slot for the
// centres of a forward slice and two environment buffers).
bool mid_sweep_zz(const tnrg_model* md) {
  if (md->xt_model != 1) return false;
  for (int b = 0; b < md->n - 1; ++b)
    if (md->zz_mask[b]) return true;
  return false;
}

GrapeLayout grape_layout(const tnrg_model* md, int K, int R, int dcap, int cs) {
  GrapeLayout g;
  const int N = md->n, M = md->m;
  g.dcap = dcap;
  g.cs = cs;
  g.nck = (M + cs - 1) / cs;
  const bool hg = mid_sweep_zz(md);
  g.nslots = g.nck + cs + 2 + (hg ? 1 : 0);
  g.nctrl = 2 * M * N + M * (N - 1);
  const size_t elems = (size_t)site_offset_slow(N, dcap, N);
  g.dims_off = align256(elems * sizeof(c2));
  g.slot_bytes = align256(g.dims_off + (size_t)(N + 1) * sizeof(int));
  g.off_x0 = (size_t)g.nslots * g.slot_bytes;
  g.off_env = g.off_x0 + align256((size_t)x_elems(dcap) * sizeof(c2));
  g.off_env2 = g.off_env + align256((size_t)(N + 1) * dcap * dcap * sizeof(c2));
  g.off_O = g.off_env2 + (hg ? align256((size_t)(N + 3) * dcap * dcap * sizeof(c2)) : 0);
  g.off_g = g.off_O + 256;
  g.off_big = align256(g.off_g + (size_t)g.nctrl * sizeof(double));
  g.traj_bytes = g.off_big + big_bytes(dcap);
  const int nt = K * R;
  g.off_flags = 0;
  g.off_stats = align256((size_t)nt * sizeof(int));
  g.off_gates = g.off_stats + align256((size_t)nt * kStats * sizeof(long long));
  g.off_traj = g.off_gates + align256((size_t)M * N * 12 * sizeof(c2));
  g.total = g.off_traj + (size_t)nt * g.traj_bytes;
  return g;
}

int default_dcap(const tnrg_model* md) {
  int half = md->n / 2;
  int c = md->chi;
  if (half < 30 && (1 << half) < c) c = 1 << half;
  return c;
}

int launch_gates(const tnrg_model* md, const double* ux, const double* uy, c2* gates,
                 hipStream_t s) {
  const int n = md->m * md->n;
  const int order = md->split_order == 1 ? 1 : 2;
  hipLaunchKernelGGL(k_gates, dim3((n + 255) / 256), dim3(256), 0, s, md->m, md->n, md->dt, order,
                     ux, uy,
                     gates);
  return TNRG_OK;
}

}  // namespace

extern "C" {

int tnrg_plan_set_threads(int32_t dcap, int32_t threads) {
  if (dcap < 1 || dcap > kMaxSites) return fail(TNRG_EINVAL, "dcap = %d out of range", dcap);
  if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512)
    return fail(TNRG_EINVAL, "threads = %d must be 0, 64, 128, 256 or 512", threads);
  if (threads == 512 && use_lds(dcap))
    return fail(TNRG_EINVAL, "512 threads only for capacities above %d", kMaxLdsCap);
  g_plan_threads[dcap].store(threads, std::memory_order_relaxed);
  return TNRG_OK;
}

int tnrg_plan_set_jacobi_lds(int32_t mode) {
  if (mode < -1 || mode > 1) return fail(TNRG_EINVAL, "jacobi_lds mode = %d must be -1, 0 or 1", mode);
  g_jacobi_lds.store(mode, std::memory_order_relaxed);
  return TNRG_OK;
}

int32_t tnrg_plan_threads(int32_t dcap) {
  if (dcap < 1 || dcap > kMaxSites) return 0;
  return threads_for_cap(dcap);
}

int32_t tnrg_bond_cap(int32_t n_sites, int32_t dcap, int32_t bond) {
  if (n_sites < 1 || dcap < 1 || bond < 0 || bond > n_sites) return 0;
  return bond_cap(n_sites, dcap, bond);
}

int64_t tnrg_mps_site_offset(int32_t n_sites, int32_t dcap, int32_t site) {
  if (n_sites < 1 || dcap < 1 || site < 0 || site > n_sites) return -1;
  return site_offset_slow(n_sites, dcap, site);
}

int64_t tnrg_mps_traj_elems(int32_t n_sites, int32_t dcap) {
  return tnrg_mps_site_offset(n_sites, dcap, n_sites);
}

const char* tnrg_last_error(void) { return g_err.c_str(); }

const char* tnrg_version(void) { return "tnrg 0.1 gfx950"; }

size_t mps_evolve_workspace_bytes(const tnrg_model* md, int32_t n_traj, int32_t dcap) {
  if (!md || n_traj < 1 || dcap < 1) return 0;
  const size_t nt = (size_t)n_traj;
  return align256(nt * sizeof(int)) + align256(nt * kStats * sizeof(long long)) +
         align256((size_t)md->m * md->n * 12 * sizeof(c2)) +
         align256(nt * (size_t)x_elems(dcap) * sizeof(c2)) + nt * big_bytes(dcap);
}

int mps_evolve(const tnrg_model* md, const double* ux, const double* uy, const double* uzz,
               const double* J, int32_t l_begin, int32_t l_end, int32_t adjoint,
               const tnrg_mps_batch* psi, void* ws, size_t ws_bytes, tnrg_stream stream) {
  ModelDev d;
  int rc = check_model(md, &d);
  if (rc) return rc;
  if ((rc = check_batch(psi, md->n, "psi"))) return rc;
  if (!ux || !uy || !uzz || !J || !ws) return fail(TNRG_EINVAL, "NULL control/crosstalk/workspace");
  if (l_begin < 0 || l_end > md->m || l_begin > l_end)
    return fail(TNRG_EINVAL, "slice range [%d, %d) outside [0, %d)", l_begin, l_end, md->m);
  const size_t need = mps_evolve_workspace_bytes(md, psi->n_traj, psi->dcap);
  if (ws_bytes < need) return fail(TNRG_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  if (psi->dcap > kMaxCap)
    return fail(TNRG_EUNSUPPORTED, "dcap = %d is above the supported %d", psi->dcap, kMaxCap);
  const bool in_lds = use_lds(psi->dcap);
  const size_t lds = in_lds ? dyn_lds_bytes(psi->dcap) : 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const size_t nt = psi->n_traj;
  EvolveArgs A;
  A.md = d;
  A.uzz = uzz;
  A.J = J;
  A.flags = reinterpret_cast<int*>(w);
  A.stats = reinterpret_cast<long long*>(w + align256(nt * sizeof(int)));
  c2* gates = reinterpret_cast<c2*>(w + align256(nt * sizeof(int)) + align256(nt * kStats * sizeof(long long)));
  A.gates = gates;
  A.x0 = reinterpret_cast<c2*>(reinterpret_cast<char*>(gates) +
                               align256((size_t)md->m * md->n * 12 * sizeof(c2)));
  A.big = reinterpret_cast<c2*>(reinterpret_cast<char*>(A.x0) +
                                align256(nt * (size_t)x_elems(psi->dcap) * sizeof(c2)));
  A.big_stride = big_bytes(psi->dcap) / sizeof(c2);
  A.data = reinterpret_cast<c2*>(psi->data);
  A.dims = psi->bond_dim;
  A.dcap = psi->dcap;
  A.stride = tnrg_mps_traj_elems(md->n, psi->dcap);
  A.l_begin = l_begin;
  A.l_end = l_end;
  A.adjoint = adjoint ? 1 : 0;
  launch_gates(md, ux, uy, gates, s);
  A.jx_elems = in_lds ? 0 : jacobi_lds_elems();
  const void* kern = in_lds ? reinterpret_cast<const void*>(lds::k_evolve)
                            : reinterpret_cast<const void*>(big::k_evolve);
  hipError_t e = hipFuncSetAttribute(
      kern, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(in_lds ? lds : (size_t)A.jx_elems * sizeof(c2)));
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_evolve)");
  if (in_lds)
    hipLaunchKernelGGL(lds::k_evolve, dim3(psi->n_traj), dim3(threads_for_cap(psi->dcap)), lds, s, A);
  else
    hipLaunchKernelGGL(big::k_evolve, dim3(psi->n_traj), dim3(threads_for_cap(psi->dcap)),
                       (size_t)A.jx_elems * sizeof(c2), s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_evolve launch");
  return TNRG_OK;
}

size_t mps_overlap_workspace_bytes(int32_t n_traj, int32_t n_sites, int32_t dcap) {
  (void)n_sites;
  if (n_traj < 1 || dcap < 1) return 0;
  return align256((size_t)n_traj * sizeof(int)) + align256((size_t)n_traj * kStats * sizeof(long long)) +
         (size_t)n_traj * big_bytes(dcap);
}

int mps_overlap(const tnrg_mps_batch* bra, const tnrg_mps_batch* ket, tnrg_c128* out, void* ws,
                size_t ws_bytes, tnrg_stream stream) {
  if (!bra || !ket) return fail(TNRG_EINVAL, "NULL batch");
  const int N = ket->n_sites;
  if (N < 2 || N > kMaxSites) return fail(TNRG_EINVAL, "n_sites = %d outside [2, %d]", N, kMaxSites);
  int rc;
  if ((rc = check_batch(bra, N, "bra"))) return rc;
  if ((rc = check_batch(ket, N, "ket"))) return rc;
  if (ket->n_traj % bra->n_traj) return fail(TNRG_EINVAL, "bra count must divide ket count");
  if (!out || !ws) return fail(TNRG_EINVAL, "NULL output/workspace");
  const int cap = std::max(bra->dcap, ket->dcap);
  if (cap > kMaxCap) return fail(TNRG_EUNSUPPORTED, "dcap = %d is above the supported %d", cap, kMaxCap);
  const size_t need = mps_overlap_workspace_bytes(ket->n_traj, N, cap);
  if (ws_bytes < need) return fail(TNRG_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  const bool in_lds = use_lds(cap);
  const size_t lds = in_lds ? dyn_lds_bytes(cap) : 0;
  OverlapArgs A;
  memset(&A, 0, sizeof A);
  A.md.N = N;
  A.bra = reinterpret_cast<const c2*>(bra->data);
  A.bdims = bra->bond_dim;
  A.bdcap = bra->dcap;
  A.bstride = tnrg_mps_traj_elems(N, bra->dcap);
  A.nb = bra->n_traj;
  A.ket = reinterpret_cast<const c2*>(ket->data);
  A.kdims = ket->bond_dim;
  A.kdcap = ket->dcap;
  A.kstride = tnrg_mps_traj_elems(N, ket->dcap);
  A.cap = cap;
  A.out = reinterpret_cast<c2*>(out);
  A.flags = static_cast<int*>(ws);
  A.big = reinterpret_cast<c2*>(static_cast<char*>(ws) + align256((size_t)ket->n_traj * sizeof(int)) +
                                align256((size_t)ket->n_traj * kStats * sizeof(long long)));
  A.big_stride = big_bytes(cap) / sizeof(c2);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const void* kern = in_lds ? reinterpret_cast<const void*>(lds::k_overlap)
                            : reinterpret_cast<const void*>(big::k_overlap);
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_overlap)");
  if (in_lds)
    hipLaunchKernelGGL(lds::k_overlap, dim3(ket->n_traj), dim3(threads_for_cap(cap)), lds, s, A);
  else
    hipLaunchKernelGGL(big::k_overlap, dim3(ket->n_traj), dim3(threads_for_cap(cap)), 0, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_overlap launch");
  return TNRG_OK;
}

size_t grape_workspace_bytes(const tnrg_model* md, int32_t K, int32_t R, int32_t dcap,
                             int32_t ckpt_stride) {
  if (!md || md->n < 2 || md->m < 1 || K < 1 || R < 1 || dcap < 0 || ckpt_stride < 0) return 0;
  const int cap = dcap > 0 ? dcap : default_dcap(md);
  const int cs = ckpt_stride > 0 ? std::min<int>(ckpt_stride, md->m)
                                 : (int)ceil(sqrt((double)md->m));
  return grape_layout(md, K, R, cap, cs).total;
}

}  // extern "C"

namespace {

// FNV-1a over the words that fix what a forward call leaves in the workspace.
struct Fnv {
  unsigned long long h = 1469598103934665603ull;
  template <class T>
  void add(const T& v) {
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
    for (size_t i = 0; i < sizeof(T); ++i) h = (h ^ p[i]) * 1099511628211ull;
  }
};

int grape_launch(int mode, const tnrg_model* md, const double* ux, const double* uy,
                 const double* uzz, int32_t K, const double* J, int32_t R,
                 const tnrg_mps_batch* inputs, const tnrg_mps_batch* targets, int32_t dcap,
                 int32_t ckpt_stride, double* F, double* g_ux, double* g_uy, double* g_uzz,
                 tnrg_c128* overlaps, tnrg_c128* traj_dO, void* ws, size_t ws_bytes,
                 tnrg_stream stream) {
  ModelDev d;
  int rc = check_model(md, &d);
  if (rc) return rc;
  if (K < 1 || R < 1) return fail(TNRG_EINVAL, "K = %d, R = %d must be >= 1", K, R);
  if (!ux || !uy || !uzz || !J) return fail(TNRG_EINVAL, "NULL controls or crosstalk");
  if (!ws) return fail(TNRG_EINVAL, "NULL workspace");
  if ((mode & kModeForward) && !F) return fail(TNRG_EINVAL, "NULL fidelity output");
  if ((mode & kModeBackward) && (!g_ux || !g_uy || !g_uzz))
    return fail(TNRG_EINVAL, "NULL gradient output");
  if ((rc = check_batch(inputs, md->n, "inputs"))) return rc;
  if ((rc = check_batch(targets, md->n, "targets"))) return rc;
  if (inputs->n_traj != R || targets->n_traj != R)
    return fail(TNRG_EINVAL, "inputs/targets must hold R = %d states", R);
  if (dcap < 0 || ckpt_stride < 0) return fail(TNRG_EINVAL, "dcap and ckpt_stride must be >= 0");
  const int cap = dcap > 0 ? dcap : default_dcap(md);
  const int cs = ckpt_stride > 0 ? std::min<int>(ckpt_stride, md->m)
                                 : (int)ceil(sqrt((double)md->m));
  const GrapeLayout G = grape_layout(md, K, R, cap, cs);
  if (ws_bytes < G.total) return fail(TNRG_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, G.total);
  if (cap > kMaxCap)
    return fail(TNRG_EUNSUPPORTED, "dcap = %d is above the supported %d", cap, kMaxCap);
  const bool in_lds = use_lds(cap);
  const size_t lds = in_lds ? dyn_lds_bytes(cap) : 0;
  if ((long long)K * R > 0x7fffffff) return fail(TNRG_EINVAL, "too many trajectories");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  GrapeArgs A;
  memset(&A, 0, sizeof A);
  A.md = d;
  A.ux = ux;
  A.uy = uy;
  A.uzz = uzz;
  A.J = J;
  A.K = K;
  A.R = R;
  A.in_data = reinterpret_cast<const c2*>(inputs->data);
  A.in_dims = inputs->bond_dim;
  A.in_dcap = inputs->dcap;
  A.in_stride = tnrg_mps_traj_elems(md->n, inputs->dcap);
  A.tg_data = reinterpret_cast<const c2*>(targets->data);
  A.tg_dims = targets->bond_dim;
  A.tg_dcap = targets->dcap;
  A.tg_stride = tnrg_mps_traj_elems(md->n, targets->dcap);
  A.dcap = cap;
  A.cs = cs;
  A.nck = G.nck;
  A.nslots = G.nslots;
  A.nctrl = G.nctrl;
  A.flags = reinterpret_cast<int*>(w + G.off_flags);
  A.stats = reinterpret_cast<long long*>(w + G.off_stats);
  c2* gates = reinterpret_cast<c2*>(w + G.off_gates);
  A.gates = gates;
  A.traj_base = w + G.off_traj;
  A.traj_bytes = G.traj_bytes;
  A.slot_bytes = G.slot_bytes;
  A.dims_off = G.dims_off;
  A.off_x0 = G.off_x0;
  A.off_env = G.off_env;
  A.off_env2 = G.off_env2;
  A.off_O = G.off_O;
  A.off_g = G.off_g;
  A.off_big = G.off_big;
  A.overlaps = reinterpret_cast<c2*>(overlaps);
  A.traj_dO = reinterpret_cast<c2*>(traj_dO);
  A.mode = mode;
  {
    Fnv f;
    f.add(md->n), f.add(md->m), f.add(md->dt), f.add(md->chi), f.add(md->trunc_eps);
    f.add(md->renormalize), f.add(d.max_sweeps), f.add(d.order), f.add(d.heis);
    for (int b = 0; b + 1 < md->n; ++b) f.add(md->zz_mask[b]), f.add(md->xt_mask[b]);
    f.add(ux), f.add(uy), f.add(uzz), f.add(J), f.add(K), f.add(R), f.add(cap), f.add(cs);
    f.add(inputs->data), f.add(targets->data), f.add(ws);
    A.tag = f.h | 1ull;  // never 0, the value of a cleared workspace
  }

  if (mode & kModeForward) launch_gates(md, ux, uy, gates, s);
  const bool mid = d.hgrad;
  const void* kern = in_lds ? (mid ? reinterpret_cast<const void*>(lds::k_grape<true>)
                                   : reinterpret_cast<const void*>(lds::k_grape<false>))
                            : (mid ? reinterpret_cast<const void*>(big::k_grape<true>)
                                   : reinterpret_cast<const void*>(big::k_grape<false>));
  A.jx_elems = in_lds ? 0 : jacobi_lds_elems();
  const size_t dyn = in_lds ? lds : (size_t)A.jx_elems * sizeof(c2);
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_grape)");
  const dim3 grid(K * R), block(threads_for_cap(cap));
  if (in_lds && mid)
    hipLaunchKernelGGL(lds::k_grape<true>, grid, block, lds, s, A);
  else if (in_lds)
    hipLaunchKernelGGL(lds::k_grape<false>, grid, block, lds, s, A);
  else if (mid)
    hipLaunchKernelGGL(big::k_grape<true>, grid, block, dyn, s, A);
  else
    hipLaunchKernelGGL(big::k_grape<false>, grid, block, dyn, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_grape launch");
  const int MN = md->m * md->n;
  const int nred = (mode & kModeBackward) ? G.nctrl : 0;
  hipLaunchKernelGGL(k_reduce, dim3(std::max(1, (nred + 255) / 256)), dim3(256), 0, s, K * R,
                     nred, MN, md->m * (md->n - 1), A.traj_base, G.traj_bytes, G.off_O, G.off_g,
                     (mode & kModeForward) ? F : nullptr, g_ux, g_uy, g_uzz);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_reduce launch");
  return TNRG_OK;
}

}  // namespace

extern "C" {

int grape_fidelity_grad(const tnrg_model* md, const double* ux, const double* uy,
                        const double* uzz, int32_t K, const double* J, int32_t R,
                        const tnrg_mps_batch* inputs, const tnrg_mps_batch* targets,
                        int32_t dcap, int32_t ckpt_stride, double* F, double* g_ux,
                        double* g_uy, double* g_uzz, tnrg_c128* overlaps, tnrg_c128* traj_dO,
                        void* ws, size_t ws_bytes, tnrg_stream stream) {
  return grape_launch(kModeForward | kModeBackward, md, ux, uy, uzz, K, J, R, inputs, targets,
                      dcap, ckpt_stride, F, g_ux, g_uy, g_uzz, overlaps, traj_dO, ws, ws_bytes,
                      stream);
}

int grape_forward(const tnrg_model* md, const double* ux, const double* uy, const double* uzz,
                  int32_t K, const double* J, int32_t R, const tnrg_mps_batch* inputs,
                  const tnrg_mps_batch* targets, int32_t dcap, int32_t ckpt_stride, double* F,
                  tnrg_c128* overlaps, void* ws, size_t ws_bytes, tnrg_stream stream) {
  return grape_launch(kModeForward, md, ux, uy, uzz, K, J, R, inputs, targets, dcap, ckpt_stride,
                      F, nullptr, nullptr, nullptr, overlaps, nullptr, ws, ws_bytes, stream);
}

int grape_backward(const tnrg_model* md, const double* ux, const double* uy, const double* uzz,
                   int32_t K, const double* J, int32_t R, const tnrg_mps_batch* inputs,
                   const tnrg_mps_batch* targets, int32_t dcap, int32_t ckpt_stride,
                   double* g_ux, double* g_uy, double* g_uzz, tnrg_c128* traj_dO, void* ws,
                   size_t ws_bytes, tnrg_stream stream) {
  return grape_launch(kModeBackward, md, ux, uy, uzz, K, J, R, inputs, targets, dcap, ckpt_stride,
                      nullptr, g_ux, g_uy, g_uzz, nullptr, traj_dO, ws, ws_bytes, stream);
}

int tnrg_status(const void* ws, int32_t n_traj, int32_t* host_flags, int64_t* stats,
                tnrg_stream stream) {
  if (!ws || n_traj < 1) return fail(TNRG_EINVAL, "NULL workspace or n_traj < 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  std::string flags((size_t)n_traj * sizeof(int), '\0');
  e = hipMemcpy(&flags[0], ws, flags.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(flags)");
  const int* f = reinterpret_cast<const int*>(flags.data());
  int any = 0;
  for (int t = 0; t < n_traj; ++t) any |= f[t];
  if (host_flags) memcpy(host_flags, f, flags.size());
  if (stats) {
    std::string st((size_t)n_traj * kStats * sizeof(long long), '\0');
    e = hipMemcpy(&st[0], static_cast<const char*>(ws) + align256((size_t)n_traj * sizeof(int)),
                  st.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(stats)");
    const long long* p = reinterpret_cast<const long long*>(st.data());
    int64_t out[18];
    memset(out, 0, sizeof out);
    for (int t = 0; t < n_traj; ++t) {
      const long long* q = p + (size_t)kStats * t;
      out[0] = std::max<int64_t>(out[0], q[0]);
      out[1] = std::max<int64_t>(out[1], q[1]);
      for (int i = 2; i < 6; ++i) out[i] += q[i];
      for (int i = 0; i < 8; ++i) out[6 + i] += q[8 + i];
      out[14] += q[6];
      out[15] += q[7];
      out[16] += q[16];
      out[17] += q[17];
    }
    memcpy(stats, out, sizeof out);
  }
  if (any & TNRG_FLAG_OVERFLOW) return fail(TNRG_EOVERFLOW, "a bond needed more than the capacity");
  if (any & TNRG_FLAG_NOCONV) return fail(TNRG_ENOCONV, "Jacobi SVD reached max_sweeps");
  if (any & TNRG_FLAG_NONFINITE) return fail(TNRG_ENONFINITE, "non-finite value met");
  if (any & TNRG_FLAG_STALE)
    return fail(TNRG_ESTALE, "grape_backward without a matching grape_forward in this workspace");
  return TNRG_OK;
}

}  // extern "C"
