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
#include "tnrg_device.hpp"

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

__global__ void k_gates(int M, int N, double dt, const double* __restrict__ ux,
                        const double* __restrict__ uy, c2* __restrict__ gates) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const double x = ux[idx], y = uy[idx];
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
// Context set-up shared by the kernels.
struct Shared {
  Layout L;
  int sdims[kMaxSites + 1];
  double red[kMaxWaves * 8];
  int sflag;
  int sk;
  double sinv;
  double sd[4];
  int si[4];
  long long sstat[kStats];
};

__device__ __forceinline__ Ctx make_ctx(Shared& sh, c2* dyn, int cap, const ModelDev& md, c2* X0) {
  Ctx C;
  C.tid = threadIdx.x;
  C.nt = blockDim.x;
  C.cap = cap;
  // buffers sized from P2 = max(4, pow2(2 cap)) so padded columns always fit
  int P2 = 4;
  while (P2 < 2 * cap) P2 <<= 1;
  const int half = P2 * P2 / 2;
  sc2* base = (sc2*)dyn;
  C.LC = base;
  C.LO = base + half;
  C.X = base + 2 * half;
  sdbl* d = (sdbl*)(C.X + P2 * (P2 + 1));
  C.sig = d;
  C.perm = (sint*)(d + P2);
  C.X0 = X0;
  C.L = (sLayout*)&sh.L;
  C.sdims = (sint*)sh.sdims;
  C.md = md;
  C.sflag = (sint*)&sh.sflag;
  C.sstat = (sll*)sh.sstat;
  C.red = (sdbl*)sh.red;
  C.sk = (sint*)&sh.sk;
  C.sinv = (sdbl*)&sh.sinv;
  C.sd = (sdbl*)sh.sd;
  C.si = (sint*)sh.si;
  if (C.tid == 0) {
    sh.sflag = 0;
    for (int q = 0; q < kStats; ++q) sh.sstat[q] = 0;
  }
  return C;
}

static size_t dyn_lds_bytes(int cap) {
  size_t P2 = 4;
  while (P2 < (size_t)2 * cap) P2 <<= 1;
  return (P2 * P2 + P2 * (P2 + 1)) * sizeof(c2) + P2 * sizeof(double) + P2 * sizeof(int);
}

// ============================================================================
// Boundary insertions (App. A): with the left environments of <b_{l+1}|a_l>
// stored, sweep right to left; at each site form the transition matrix
// rho_j[s][s'] = <b|(|s><s'|)_j|a> and, on bonds with a u^zz control, the
// two-site element of (R Z R^dag) (x) (R Z R^dag); accumulate
//   outer half of slice l   (l >= 1):    G = dR R^dag
//   inner half of slice l+1 (l <= M-1):  G = R^dag dR
//   ZZ control of slice l   (l >= 1):    -i dt <b|W_b W_{b+1}|a>
// into the trajectory's gradient as 2 Re(conj(O) dO) (and dO itself when
// requested).  lb is the 1-based boundary index l = 0..M.
struct GradOut {
  double* g;  // [nctrl] 2 Re(conj O dO)
  c2* dO;     // [nctrl] or nullptr
  c2 O;
};

__device__ __forceinline__ void right_insertions(Ctx& C, const c2* bra, const int* bd, const c2* ket,
                                 const int* kd, const sLayout& L, const c2* envs, int lb,
                                 const c2* gates, GradOut go) {
  const int N = C.md.N, M = C.md.M;
  const int cc = C.cap * C.cap;
  const double dt = C.md.dt;
  EnvBufs eb = env_bufs(C);
  sc2* TF = eb.TF;
  sc2* TFp = eb.TFp;
  sc2* Tq = C.LO;  // two-site intermediate (2 cap^2)
  if (C.tid == 0) eb.F[0] = cmk(1.0, 0.0);
  __syncthreads();
  for (int j = N - 1; j >= 0; --j) {
    const int bl = bd[j], br = bd[j + 1], al = kd[j], ar = kd[j + 1];
    const c2* A = ket + L.off[j];
    const c2* Bt = bra + L.off[j];
    const int rc = L.cap[j + 1];
    for (int idx = C.tid; idx < bl * al; idx += C.nt) eb.E[idx] = envs[(size_t)j * cc + idx];
    if (C.tid == 0) C.sstat[5] += 16LL * (al * br * ar + bl * br * al + al * bl * br);
    // TF[s'][a][x] = sum_y A[a,s',y] F[y][x]     (al x br)
    for (int idx = C.tid; idx < 2 * al * br; idx += C.nt) {
      const int s = idx / (al * br);
      const int rem = idx - s * al * br;
      const int a = rem / br, x = rem - a * br;
      c2 acc = cmk(0.0, 0.0);
      for (int y = 0; y < ar; ++y) acc = cfma(A[(size_t)(a * 2 + s) * rc + y], eb.F[y * br + x], acc);
      TF[s * cc + a * br + x] = acc;
    }
    __syncthreads();
    // rho[s][s'] = sum_{z,x} conj(B[z,s,x]) sum_a E[z][a] TF[s'][a][x]
    c2 rho[4] = {cmk(0, 0), cmk(0, 0), cmk(0, 0), cmk(0, 0)};
    for (int idx = C.tid; idx < bl * br; idx += C.nt) {
      const int z = idx / br, x = idx - z * br;
      c2 u0 = cmk(0.0, 0.0), u1 = cmk(0.0, 0.0);
      for (int a = 0; a < al; ++a) {
        const c2 e = eb.E[z * al + a];
        u0 = cfma(e, TF[a * br + x], u0);
        u1 = cfma(e, TF[cc + a * br + x], u1);
      }
      const c2 b0 = Bt[(size_t)(z * 2 + 0) * rc + x];
      const c2 b1 = Bt[(size_t)(z * 2 + 1) * rc + x];
      rho[0] = cfmac(b0, u0, rho[0]);
      rho[1] = cfmac(b0, u1, rho[1]);
      rho[2] = cfmac(b1, u0, rho[2]);
      rho[3] = cfmac(b1, u1, rho[3]);
    }
    block_sum<4>(C, rho);
    // F_j[a][z] = sum_s sum_x TF[s][a][x] conj(B[z,s,x])   (al x bl)
    for (int idx = C.tid; idx < al * bl; idx += C.nt) {
      const int a = idx / bl, z = idx - a * bl;
      c2 acc = cmk(0.0, 0.0);
      for (int s = 0; s < 2; ++s)
        for (int x = 0; x < br; ++x)
          acc = cfmac(Bt[(size_t)(z * 2 + s) * rc + x], TF[s * cc + a * br + x], acc);
      eb.F[idx] = acc;
    }
    // two-site element on a controlled bond j (needs site j+1 and TFp)
    const bool zz = (lb >= 1) && (j <= N - 2) && bit(C.md.zzm, j);
    c2 val = cmk(0.0, 0.0);
    if (zz) {
      const int s0 = lb - 1;
      const M22 R1 = m22_load(gate_ptr(gates, N, s0, j));
      const M22 R2 = m22_load(gate_ptr(gates, N, s0, j + 1));
      M22 Zm;
      Zm.m[0] = cmk(1, 0); Zm.m[1] = cmk(0, 0); Zm.m[2] = cmk(0, 0); Zm.m[3] = cmk(-1, 0);
      const M22 W1 = m22_mul(m22_mul(R1, Zm), m22_dag(R1));
      const M22 W2 = m22_mul(m22_mul(R2, Zm), m22_dag(R2));
      // Tq[t][z][y] = sum_w E[z][w] A[w,t,y]      (bl x ar)
      for (int idx = C.tid; idx < 2 * bl * ar; idx += C.nt) {
        const int t = idx / (bl * ar);
        const int rem = idx - t * bl * ar;
        const int z = rem / ar, y = rem - z * ar;
        c2 acc = cmk(0.0, 0.0);
        for (int w = 0; w < al; ++w) acc = cfma(eb.E[z * al + w], A[(size_t)(w * 2 + t) * rc + y], acc);
        Tq[t * cc + z * ar + y] = acc;
      }
      __syncthreads();
      // E'[x][y] = sum_{s,t} W1[s][t] sum_z conj(B[z,s,x]) Tq[t][z][y]   (br x ar) -> E
      for (int idx = C.tid; idx < br * ar; idx += C.nt) {
        const int x = idx / ar, y = idx - x * ar;
        c2 acc = cmk(0.0, 0.0);
        for (int s = 0; s < 2; ++s) {
          for (int t = 0; t < 2; ++t) {
            c2 inner = cmk(0.0, 0.0);
            for (int z = 0; z < bl; ++z)
              inner = cfmac(Bt[(size_t)(z * 2 + s) * rc + x], Tq[t * cc + z * ar + y], inner);
            acc = cfma(W1.m[2 * s + t], inner, acc);
          }
        }
        eb.E[idx] = acc;
      }
      __syncthreads();
      // rho'(s,t) on site j+1 with E' and TFp = A_{j+1} F_{j+2}
      const int bl2 = br, br2 = bd[j + 2], al2 = ar;
      const c2* B2 = bra + L.off[j + 1];
      const int rc2 = L.cap[j + 2];
      c2 rp[4] = {cmk(0, 0), cmk(0, 0), cmk(0, 0), cmk(0, 0)};
      for (int idx = C.tid; idx < bl2 * br2; idx += C.nt) {
        const int z = idx / br2, x = idx - z * br2;
        c2 u0 = cmk(0.0, 0.0), u1 = cmk(0.0, 0.0);
        for (int a = 0; a < al2; ++a) {
          const c2 e = eb.E[z * al2 + a];
          u0 = cfma(e, TFp[a * br2 + x], u0);
          u1 = cfma(e, TFp[cc + a * br2 + x], u1);
        }
        const c2 b0 = B2[(size_t)(z * 2 + 0) * rc2 + x];
        const c2 b1 = B2[(size_t)(z * 2 + 1) * rc2 + x];
        rp[0] = cfmac(b0, u0, rp[0]);
        rp[1] = cfmac(b0, u1, rp[1]);
        rp[2] = cfmac(b1, u0, rp[2]);
        rp[3] = cfmac(b1, u1, rp[3]);
      }
      block_sum<4>(C, rp);
      for (int q = 0; q < 4; ++q) val = cfma(W2.m[q], rp[q], val);
    }
    if (C.tid == 0) {
      auto tr = [&](const M22& G) {
        c2 v = cmk(0.0, 0.0);
        for (int q = 0; q < 4; ++q) v = cfma(G.m[q], rho[q], v);
        return v;
      };
      auto add = [&](size_t idx, c2 v) {
        go.g[idx] += 2.0 * (go.O.x * v.x + go.O.y * v.y);
        if (go.dO) go.dO[idx] = cadd(go.dO[idx], v);
      };
      const size_t MN = (size_t)M * N;
      if (lb >= 1) {
        const int s0 = lb - 1;
        const c2* gp = gate_ptr(gates, N, s0, j);
        const M22 R = m22_load(gp), dx = m22_load(gp + 4), dy = m22_load(gp + 8);
        const M22 Rd = m22_dag(R);
        add((size_t)s0 * N + j, tr(m22_mul(dx, Rd)));
        add(MN + (size_t)s0 * N + j, tr(m22_mul(dy, Rd)));
      }
      if (lb <= M - 1) {
        const int s0 = lb;
        const c2* gp = gate_ptr(gates, N, s0, j);
        const M22 R = m22_load(gp), dx = m22_load(gp + 4), dy = m22_load(gp + 8);
        const M22 Rd = m22_dag(R);
        add((size_t)s0 * N + j, tr(m22_mul(Rd, dx)));
        add(MN + (size_t)s0 * N + j, tr(m22_mul(Rd, dy)));
      }
      if (zz) {
        const int s0 = lb - 1;
        // -i dt val
        add(2 * MN + (size_t)s0 * (N - 1) + j, cmk(dt * val.y, -dt * val.x));
      }
    }
    __syncthreads();
    sc2* tmp = TF;
    TF = TFp;
    TFp = tmp;
  }
}

// ============================================================================
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
  c2* overlaps;
  c2* traj_dO;
  int mode;                // kModeForward | kModeBackward
  unsigned long long tag;  // fingerprint of the call's arguments
};

constexpr int kModeForward = 1, kModeBackward = 2;

// Adjoint sweep of one trajectory (App. A): insertions at boundary M with the
// environments `envs` already built for <T|a_M>, then for l = M-1 .. 0 the
// backward state b_{l+1} = U_{l+1}^dag b_{l+2} and the insertions at the
// boundary pair (b_{l+1}, a_l), the a_l recomputed segment by segment from
// the checkpoints a_0, a_cs, a_2cs, ...
__device__ __forceinline__ void grape_adjoint(Ctx& C, const GrapeArgs& A, char* base, GradOut& go,
                                              c2* envs, const double* Jrow, const sLayout& L) {
  const int M = A.md.M;
  auto slot = [&](int s) { return reinterpret_cast<c2*>(base + (size_t)s * A.slot_bytes); };
  auto sdim = [&](int s) {
    return reinterpret_cast<int*>(base + (size_t)s * A.slot_bytes + A.dims_off);
  };
  const int s_seg = A.nck, s_aM = A.nck + A.cs - 1, s_b = A.nck + A.cs + 1;
  long long te = ph_now(C);
  right_insertions(C, slot(s_b), sdim(s_b), slot(s_aM), sdim(s_aM), L, envs, M, A.gates, go);
  ph_add(C, kPhEnvR, te);
  adjoint_slice(C, slot(s_b), sdim(s_b), slot(s_b), sdim(s_b), A.gates, M - 1, A.uzz, Jrow);
  for (int i = A.nck - 1; i >= 0; --i) {
    const int L0 = i * A.cs;
    const int L1 = min((i + 1) * A.cs, M) - 1;
    for (int l = L0 + 1; l <= L1; ++l) {
      const int src = (l - 1 == L0) ? i : s_seg + (l - 2 - L0);
      const int dst = s_seg + (l - 1 - L0);
      forward_slice(C, slot(src), sdim(src), slot(dst), sdim(dst), A.gates, l - 1, A.uzz, Jrow);
    }
    for (int l = L1; l >= L0; --l) {
      const int ket = (l == L0) ? i : s_seg + (l - 1 - L0);
      te = ph_now(C);
      left_envs(C, slot(s_b), sdim(s_b), L, slot(ket), sdim(ket), L, envs);
      ph_add(C, kPhEnvL, te);
      right_insertions(C, slot(s_b), sdim(s_b), slot(ket), sdim(ket), L, envs, l, A.gates, go);
      ph_add(C, kPhEnvR, te);
      if (l >= 1)
        adjoint_slice(C, slot(s_b), sdim(s_b), slot(s_b), sdim(s_b), A.gates, l - 1, A.uzz, Jrow);
    }
  }
}

__global__ void __launch_bounds__(256) k_grape(GrapeArgs A) {
  extern __shared__ __align__(16) c2 dyn[];
  __shared__ Shared sh;
  const int t = blockIdx.x;
  const int k = t / A.R, r = t % A.R;
  const int N = A.md.N, M = A.md.M;
  char* base = A.traj_base + (size_t)t * A.traj_bytes;
  Ctx C = make_ctx(sh, dyn, A.dcap, A.md, reinterpret_cast<c2*>(base + A.off_x0));
  layout_build(*(sLayout*)&sh.L, N, A.dcap);
  const sLayout& L = *(sLayout*)&sh.L;
  long long t_all = ph_now(C);
  auto slot = [&](int s) { return reinterpret_cast<c2*>(base + (size_t)s * A.slot_bytes); };
  auto sdim = [&](int s) {
    return reinterpret_cast<int*>(base + (size_t)s * A.slot_bytes + A.dims_off);
  };
  const int s_seg = A.nck, s_aM = A.nck + A.cs - 1, s_work = A.nck + A.cs, s_b = A.nck + A.cs + 1;
  const double* Jrow = A.J + (size_t)k * (N - 1);
  c2* envs = reinterpret_cast<c2*>(base + A.off_env);
  double* g = reinterpret_cast<double*>(base + A.off_g);
  c2* dO = A.traj_dO ? A.traj_dO + (size_t)t * A.nctrl : nullptr;
  const bool fwd = A.mode & kModeForward, bwd = A.mode & kModeBackward;
  unsigned long long* tagp = reinterpret_cast<unsigned long long*>(base + A.off_O + sizeof(c2));

  if (!fwd) {
    // the adjoint sweep reads the checkpoints a forward call with the same
    // arguments left in this workspace; it also keeps that call's flags and
    // counters and adds its own
    if (C.tid == 0) {
      if (*tagp == A.tag) {
        sh.sflag = A.flags[t] & ~TNRG_FLAG_STALE;
        for (int q = 0; q < kStats; ++q) sh.sstat[q] = A.stats[(size_t)t * kStats + q];
      } else {
        sh.sflag = TNRG_FLAG_STALE;
      }
    }
  }
  if (bwd) {
    for (int i = C.tid; i < A.nctrl; i += C.nt) {
      g[i] = 0.0;
      if (dO) dO[i] = cmk(0.0, 0.0);
    }
  }
  __syncthreads();
  if (!(sh.sflag & TNRG_FLAG_STALE)) {
    copy_mps(C, A.tg_data + (size_t)r * A.tg_stride, A.tg_dims + (size_t)r * (N + 1), A.tg_dcap,
             slot(s_b), sdim(s_b), L);
    if (fwd) {
      copy_mps(C, A.in_data + (size_t)r * A.in_stride, A.in_dims + (size_t)r * (N + 1),
               A.in_dcap, slot(0), sdim(0), L);
      // forward pass with checkpoints a_0, a_cs, a_2cs, ...
      int cur = 0;
      for (int l = 0; l < M; ++l) {
        int dst;
        if (l + 1 == M)
          dst = s_aM;
        else if ((l + 1) % A.cs == 0)
          dst = (l + 1) / A.cs;
        else
          dst = s_work;
        forward_slice(C, slot(cur), sdim(cur), slot(dst), sdim(dst), A.gates, l, A.uzz, Jrow);
        cur = dst;
      }
    }
    // boundary M: O = <T|a_M> (recomputed bit for bit by a backward-only call)
    GradOut go;
    go.g = g;
    go.dO = dO;
    long long te = ph_now(C);
    go.O = left_envs(C, slot(s_b), sdim(s_b), L, slot(s_aM), sdim(s_aM), L, envs);
    ph_add(C, kPhEnvL, te);
    if (fwd && C.tid == 0) {
      *reinterpret_cast<c2*>(base + A.off_O) = go.O;
      *tagp = A.tag;
      if (A.overlaps) A.overlaps[t] = go.O;
    }
    if (bwd) grape_adjoint(C, A, base, go, envs, Jrow, L);
  }
  __syncthreads();
  ph_add(C, kPhTotal, t_all);
  if (C.tid == 0) {
    A.flags[t] = sh.sflag;
    for (int q = 0; q < kStats; ++q) A.stats[(size_t)t * kStats + q] = sh.sstat[q];
  }
}

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

// ============================================================================
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
  int* flags;
  long long* stats;
};

__global__ void __launch_bounds__(256) k_evolve(EvolveArgs A) {
  extern __shared__ __align__(16) c2 dyn[];
  __shared__ Shared sh;
  const int t = blockIdx.x;
  const int N = A.md.N;
  const int cap = A.dcap;
  Ctx C = make_ctx(sh, dyn, cap, A.md, A.x0 + (size_t)t * x_elems(cap));
  layout_build(*(sLayout*)&sh.L, N, cap);
  c2* psi = A.data + (size_t)t * A.stride;
  int* d = A.dims + (size_t)t * (N + 1);
  const double* Jrow = A.J + (size_t)t * (N - 1);
  for (int b = C.tid; b <= N; b += C.nt) {
    const int db = d[b];
    if (db > sh.L.cap[b] || db < 1 || ((b == 0 || b == N) && db != 1)) flag_or(C, 1);
  }
  __syncthreads();
  if (!sh.sflag) {
    if (!A.adjoint) {
      for (int l = A.l_begin; l < A.l_end; ++l) forward_slice(C, psi, d, psi, d, A.gates, l, A.uzz, Jrow);
    } else {
      for (int l = A.l_end - 1; l >= A.l_begin; --l)
        adjoint_slice(C, psi, d, psi, d, A.gates, l, A.uzz, Jrow);
    }
  }
  __syncthreads();
  if (C.tid == 0) {
    A.flags[t] = sh.sflag;
    for (int q = 0; q < kStats; ++q) A.stats[(size_t)t * kStats + q] = sh.sstat[q];
  }
}

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
};

__global__ void __launch_bounds__(256) k_overlap(OverlapArgs A) {
  extern __shared__ __align__(16) c2 dyn[];
  __shared__ Shared sh;
  __shared__ Layout L2;
  const int t = blockIdx.x;
  const int N = A.md.N;
  Ctx C = make_ctx(sh, dyn, A.cap, A.md, nullptr);
  layout_build(*(sLayout*)&sh.L, N, A.kdcap);
  layout_build(*(sLayout*)&L2, N, A.bdcap);
  const int rb = t % A.nb;
  const c2 o = left_envs(C, A.bra + (size_t)rb * A.bstride, A.bdims + (size_t)rb * (N + 1), *(sLayout*)&L2,
                         A.ket + (size_t)t * A.kstride, A.kdims + (size_t)t * (N + 1), *(sLayout*)&sh.L,
                         nullptr);
  if (C.tid == 0) {
    A.out[t] = o;
    A.flags[t] = 0;
  }
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
  for (int b = 0; b < md->n - 1; ++b) {
    if (md->zz_mask[b]) d.zzm[b >> 6] |= 1ull << (b & 63);
    if (md->xt_mask[b]) d.xtm[b >> 6] |= 1ull << (b & 63);
  }
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

// Fewest threads for capacity cap: every Jacobi round processes up to cap
// column pairs with at least pow2(2 cap) / 8 lanes each (8 rows per lane).
int min_threads(int cap) {
  int p2 = 1;
  while (p2 < 2 * cap) p2 <<= 1;
  const int need = (p2 / 8 > 1 ? p2 / 8 : 1) * cap;
  int nt = 64;
  while (nt < need) nt *= 2;
  return nt;
}

int default_threads(int cap) { return min_threads(cap); }

int threads_for_cap(int cap) {
  if (cap >= 0 && cap <= kMaxSites) {
    const int t = g_plan_threads[cap].load(std::memory_order_relaxed);
    if (t >= min_threads(cap)) return t;
  }
  return default_threads(cap);
}

// Largest dynamic LDS a workgroup may use on gfx950.
constexpr size_t kMaxDynLds = 160 * 1024 - sizeof(Shared) - 512;
// The bond update keeps a (2 cap) x (2 cap) problem inside one wave's lane
// range for its pivot search and sort.
constexpr int kMaxCap = 32;

struct GrapeLayout {
  int cs, nck, nslots, nctrl, dcap;
  size_t slot_bytes, dims_off, off_x0, off_env, off_O, off_g, traj_bytes;
  size_t off_flags, off_stats, off_gates, off_traj, total;
};

GrapeLayout grape_layout(const tnrg_model* md, int K, int R, int dcap, int cs) {
  GrapeLayout g;
  const int N = md->n, M = md->m;
  g.dcap = dcap;
  g.cs = cs;
  g.nck = (M + cs - 1) / cs;
  g.nslots = g.nck + cs + 2;
  g.nctrl = 2 * M * N + M * (N - 1);
  const size_t elems = (size_t)site_offset_slow(N, dcap, N);
  g.dims_off = align256(elems * sizeof(c2));
  g.slot_bytes = align256(g.dims_off + (size_t)(N + 1) * sizeof(int));
  g.off_x0 = (size_t)g.nslots * g.slot_bytes;
  g.off_env = g.off_x0 + align256((size_t)x_elems(dcap) * sizeof(c2));
  g.off_O = g.off_env + align256((size_t)(N + 1) * dcap * dcap * sizeof(c2));
  g.off_g = g.off_O + 256;
  g.traj_bytes = align256(g.off_g + (size_t)g.nctrl * sizeof(double));
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
  hipLaunchKernelGGL(k_gates, dim3((n + 255) / 256), dim3(256), 0, s, md->m, md->n, md->dt, ux, uy,
                     gates);
  return TNRG_OK;
}

}  // namespace

extern "C" {

int tnrg_plan_set_threads(int32_t dcap, int32_t threads) {
  if (dcap < 1 || dcap > kMaxSites) return fail(TNRG_EINVAL, "dcap = %d out of range", dcap);
  if (threads != 0 && threads != 64 && threads != 128 && threads != 256)
    return fail(TNRG_EINVAL, "threads = %d must be 0, 64, 128 or 256", threads);
  g_plan_threads[dcap].store(threads, std::memory_order_relaxed);
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
         nt * (size_t)x_elems(dcap) * sizeof(c2);
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
  const size_t lds = dyn_lds_bytes(psi->dcap);
  if (lds > kMaxDynLds || psi->dcap > kMaxCap)
    return fail(TNRG_EUNSUPPORTED, "dcap = %d is above the supported %d", psi->dcap, kMaxCap);
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
  A.data = reinterpret_cast<c2*>(psi->data);
  A.dims = psi->bond_dim;
  A.dcap = psi->dcap;
  A.stride = tnrg_mps_traj_elems(md->n, psi->dcap);
  A.l_begin = l_begin;
  A.l_end = l_end;
  A.adjoint = adjoint ? 1 : 0;
  launch_gates(md, ux, uy, gates, s);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_evolve),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_evolve)");
  hipLaunchKernelGGL(k_evolve, dim3(psi->n_traj), dim3(threads_for_cap(psi->dcap)), lds, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_evolve launch");
  return TNRG_OK;
}

size_t mps_overlap_workspace_bytes(int32_t n_traj, int32_t n_sites, int32_t dcap) {
  (void)n_sites;
  (void)dcap;
  if (n_traj < 1) return 0;
  return align256((size_t)n_traj * sizeof(int)) + align256((size_t)n_traj * kStats * sizeof(long long));
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
  const size_t need = mps_overlap_workspace_bytes(ket->n_traj, N, ket->dcap);
  if (ws_bytes < need) return fail(TNRG_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need);
  const int cap = std::max(bra->dcap, ket->dcap);
  const size_t lds = dyn_lds_bytes(cap);
  if (lds > kMaxDynLds) return fail(TNRG_EUNSUPPORTED, "dcap = %d needs %zu bytes of LDS", cap, lds);
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
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_overlap),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_overlap)");
  hipLaunchKernelGGL(k_overlap, dim3(ket->n_traj), dim3(threads_for_cap(cap)), lds, s, A);
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
  const size_t lds = dyn_lds_bytes(cap);
  if (lds > kMaxDynLds || cap > kMaxCap)
    return fail(TNRG_EUNSUPPORTED, "dcap = %d is above the supported %d", cap, kMaxCap);
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
  A.off_O = G.off_O;
  A.off_g = G.off_g;
  A.overlaps = reinterpret_cast<c2*>(overlaps);
  A.traj_dO = reinterpret_cast<c2*>(traj_dO);
  A.mode = mode;
  {
    Fnv f;
    f.add(md->n), f.add(md->m), f.add(md->dt), f.add(md->chi), f.add(md->trunc_eps);
    f.add(md->renormalize), f.add(d.max_sweeps);
    for (int b = 0; b + 1 < md->n; ++b) f.add(md->zz_mask[b]), f.add(md->xt_mask[b]);
    f.add(ux), f.add(uy), f.add(uzz), f.add(J), f.add(K), f.add(R), f.add(cap), f.add(cs);
    f.add(inputs->data), f.add(targets->data), f.add(ws);
    A.tag = f.h | 1ull;  // never 0, the value of a cleared workspace
  }

  if (mode & kModeForward) launch_gates(md, ux, uy, gates, s);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_grape),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_grape)");
  hipLaunchKernelGGL(k_grape, dim3(K * R), dim3(threads_for_cap(cap)), lds, s, A);
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
