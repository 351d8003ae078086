// Memory-space independent building blocks of the MPS robust-GRAPE hot path
// for gfx950: complex arithmetic, 2x2 gates, the model and MPS layout seen by
// the kernels, and wave-level DPP reductions.
//
// Method references (Le, Mintert, Ginossar): second-order slice of Sec. II,
// Eq. 4 with SVD compression to a maximum bond size; ensemble state fidelity
// of Sec. II, Eq. 7; adjoint gradient of App. A, Eqs. A1-A2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnrg {


// Complex double as a clang vector of two doubles (x = real, y = imaginary):
// a builtin type, usable in every address space, 16-byte aligned like the
// {re, im} storage of complex128.
typedef double c2 __attribute__((ext_vector_type(2)));

constexpr int kMaxSites = 256;
constexpr int kStats = 24;
enum { kPhLoad = 8, kPhTheta, kPhLQ, kPhJacobi, kPhFinish, kPhEnvL, kPhEnvR, kPhTotal,
       kPhJacRounds = 16, kPhJacSweepEnd };
constexpr int kMaxWaves = 16;

// ----------------------------------------------------------------------------
// complex helpers (x = real, y = imaginary)
__device__ __forceinline__ c2 cmk(double r, double i) {
  c2 v;
  v.x = r;
  v.y = i;
  return v;
}
__device__ __forceinline__ c2 cadd(c2 a, c2 b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c2 csub(c2 a, c2 b) { return cmk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ c2 cconj(c2 a) { return cmk(a.x, -a.y); }
__device__ __forceinline__ c2 cscale(c2 a, double s) { return cmk(a.x * s, a.y * s); }
__device__ __forceinline__ c2 cmul(c2 a, c2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
__device__ __forceinline__ c2 cfma(c2 a, c2 b, c2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a) * b
__device__ __forceinline__ c2 cfmac(c2 a, c2 b, c2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double cabs2(c2 a) { return fma(a.x, a.x, a.y * a.y); }

// ----------------------------------------------------------------------------
// Complex matrix product on the fp64 matrix cores:
//   out(i, j) = sum_q a(i, q) b(q, j),   i < m, j < n, q < kd
// in 16 x 16 output tiles, one tile per wave at a time (tile t on wave
// t mod waves), q in steps of 4 through v_mfma_f64_16x16x4f64.  The complex
// product takes three real products per step (Gauss): P1 = ar br,
// P2 = ai bi, P3 = (ar + ai)(br + bi); re = P1 - P2, im = P3 - P1 - P2.
// The operands of kSteps steps are loaded before their products are
// issued, so a tile waits for memory once per 4 kSteps of depth.  Operand layout of
// the instruction: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of
// the 16 x 4 and 4 x 16 blocks; item v of lane l holds C[4 v + l / 16][l % 16].
// Out-of-range operands are read as zero (fa, fb are only called in range),
// fs(i, j, value) is called once per output element in range.  The summation
// order of an element depends only on kd, never on the thread count.  Every
// thread of the workgroup calls it (nt a multiple of 64); no barrier inside.
typedef double v4d __attribute__((ext_vector_type(4)));
template <int kSteps, class FA, class FB, class FS>
__device__ __forceinline__ void cgemm_mfma(int tid, int nt, int m, int n, int kd, FA fa, FB fb,
                                           FS fs) {
  const int lane = tid & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int tn = (n + 15) >> 4;
  const int ntile = ((m + 15) >> 4) * tn;
  for (int t = tid >> 6; t < ntile; t += nt >> 6) {
    const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
    const int ia = i0 + li, jb = j0 + li;
    const bool arow = ia < m, bcol = jb < n;
    v4d p1 = {0.0, 0.0, 0.0, 0.0}, p2 = {0.0, 0.0, 0.0, 0.0}, p3 = {0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < kd; q0 += 4 * kSteps) {
      c2 a[kSteps], b[kSteps];
#pragma unroll
      for (int u = 0; u < kSteps; ++u) {
        const int q = q0 + 4 * u + lq;
        a[u] = (arow && q < kd) ? fa(ia, q) : cmk(0.0, 0.0);
        b[u] = (q < kd && bcol) ? fb(q, jb) : cmk(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < kSteps; ++u) {
        if (q0 + 4 * u < kd) {  // uniform across the wave
          p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u].x, p1, 0, 0, 0);
          p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, b[u].y, p2, 0, 0, 0);
          p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x + a[u].y, b[u].x + b[u].y, p3, 0, 0, 0);
        }
      }
    }
    if (bcol) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 4 * v + lq;
        if (i < m) fs(i, jb, cmk(p1[v] - p2[v], p3[v] - p1[v] - p2[v]));
      }
    }
  }
}

// 2x2 complex matrix, row-major g[s][t] = m[2*s+t]
struct M22 {
  c2 m[4];
};
__device__ __forceinline__ M22 m22_load(const c2* p) {
  M22 r;
  r.m[0] = p[0]; r.m[1] = p[1]; r.m[2] = p[2]; r.m[3] = p[3];
  return r;
}
__device__ __forceinline__ M22 m22_dag(const M22& a) {
  M22 r;
  r.m[0] = cconj(a.m[0]); r.m[1] = cconj(a.m[2]);
  r.m[2] = cconj(a.m[1]); r.m[3] = cconj(a.m[3]);
  return r;
}
// Row s of G applied to (x0, x1): G[s][0] x0 + G[s][1] x1, with selects
// instead of a dynamically indexed register array.
__device__ __forceinline__ c2 m22_row(const M22& G, int s, c2 x0, c2 x1) {
  const c2 g0 = s ? G.m[2] : G.m[0];
  const c2 g1 = s ? G.m[3] : G.m[1];
  return cfma(g1, x1, cmul(g0, x0));
}
__device__ __forceinline__ M22 m22_mul(const M22& a, const M22& b) {
  M22 r;
  r.m[0] = cadd(cmul(a.m[0], b.m[0]), cmul(a.m[1], b.m[2]));
  r.m[1] = cadd(cmul(a.m[0], b.m[1]), cmul(a.m[1], b.m[3]));
  r.m[2] = cadd(cmul(a.m[2], b.m[0]), cmul(a.m[3], b.m[2]));
  r.m[3] = cadd(cmul(a.m[2], b.m[1]), cmul(a.m[3], b.m[3]));
  return r;
}

// ----------------------------------------------------------------------------
// Problem statement as seen by the kernels (passed by value).
struct ModelDev {
  int N, M;
  double dt;
  int chi;
  double eps;
  int renorm;
  int max_sweeps;
  int profile;      // 1: accumulate phase clock ticks into the stats
  int order;        // Trotter split: 2 (R Z R) or 1 (X Y Z)
  int heis;         // 1: Heisenberg crosstalk J^x XX + J^y YY + J^z ZZ, J row [N-1][3]
  int hgrad;        // heis and some bond carries u^zz: mid-sweep u^zz insertions
  int zz_lo, zz_hi; // lowest and highest bond with u^zz (N-1, -1 when none)
  uint64_t zzm[4];  // bit b: bond b carries u^zz
  uint64_t xtm[4];  // bit b: bond b carries crosstalk J
};
// Two-site gate exp(-i t (jx XX + jy YY + cz ZZ)) of one bond (Sec. III,
// Eq. 9).  The three terms commute and couple |s s'> only with
// |1-s 1-s'>, so the gate is block diagonal.  On {|00>, |11>} (block 0)
// ZZ = +1 and XX + YY acts as (jx - jy) sigma_x, so the block is
// e^{-i t cz} (cos(a) I - i sin(a) sigma_x) with a = t (jx - jy); on
// {|01>, |10>} (block 1) ZZ = -1 and the block is e^{+i t cz} times the same
// form with a = t (jx + jy).  d = diagonal, o = off-diagonal entry of each
// block.  With jx = jy = 0 it is the ZZ phase (o = 0 exactly).
struct BondGate {
  c2 d[2], o[2];
};
__device__ __forceinline__ BondGate bond_gate(double t, double jx, double jy, double cz) {
  BondGate g;
  const double z = t * cz, a0 = t * (jx - jy), a1 = t * (jx + jy);
  const double cp = cos(z), sp = sin(z);
  const c2 p0 = cmk(cp, -sp), p1 = cmk(cp, sp);
  const double c0 = cos(a0), s0 = sin(a0), c1 = cos(a1), s1 = sin(a1);
  g.d[0] = cmk(p0.x * c0, p0.y * c0);
  g.o[0] = cmk(p0.y * s0, -p0.x * s0);  // p0 (-i s0)
  g.d[1] = cmk(p1.x * c1, p1.y * c1);
  g.o[1] = cmk(p1.y * s1, -p1.x * s1);
  return g;
}

__device__ __forceinline__ bool bit(const uint64_t* m, int b) {
  // every word is read and the choice is made on values, never on an
  // address, so the mask words (and the context holding them) stay in
  // registers
  const uint64_t w0 = m[0], w1 = m[1], w2 = m[2], w3 = m[3];
  const int k = b >> 6;
  uint64_t w = w0;
  w = k == 1 ? w1 : w;
  w = k == 2 ? w2 : w;
  w = k == 3 ? w3 : w;
  return (w >> (b & 63)) & 1ull;
}

// Capacity of bond b: min(dcap, 2^b, 2^(N-b)).
__host__ __device__ __forceinline__ int bond_cap(int N, int dcap, int b) {
  int c = dcap;
  if (b < 30 && (1 << b) < c) c = 1 << b;
  int rb = N - b;
  if (rb < 30 && (1 << rb) < c) c = 1 << rb;
  return c;
}

// Elements of the Jacobi working matrix for capacity cap: P2 (P2 + 1) with
// P2 = max(4, pow2(2 cap)) (padded columns plus one element of bank skew).
__host__ __device__ inline long long x_elems(int cap) {
  long long p = 4;
  while (p < 2LL * cap) p <<= 1;
  return p * (p + 1);
}

// Fixed-capacity MPS layout, built in LDS at kernel start.
struct Layout {
  int N;
  int dcap;
  int cap[kMaxSites + 1];
  long long off[kMaxSites + 1];  // off[N] = elements per trajectory
};
__host__ __device__ inline long long site_offset_slow(int N, int dcap, int j) {
  long long o = 0;
  for (int i = 0; i < j; ++i) o += (long long)bond_cap(N, dcap, i) * 2 * bond_cap(N, dcap, i + 1);
  return o;
}

// ----------------------------------------------------------------------------
// Butterfly sums over aligned groups of G lanes (G = 1, 2, 4, 8, 16) with DPP
// lane permutations.  Every step combines a lane with the partner of an
// involution (row mirror, half-row mirror, xor 1, xor 2) as a + b on one side
// and b + a on the other, so all G lanes end with bit-identical sums.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7-i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15-i within 16

// Inactive steps add +0 through a select instead of a branch, so the
// reductions of several independent values interleave.
__device__ __forceinline__ double group_sum(double v, int G) {
  v += (G >= 16) ? dpp_d<kDppMirror>(v) : 0.0;
  v += (G >= 8) ? dpp_d<kDppHalfMirror>(v) : 0.0;
  v += (G >= 2) ? dpp_d<kDppXor1>(v) : 0.0;
  v += (G >= 4) ? dpp_d<kDppXor2>(v) : 0.0;
  return v;
}

// Groups of 32 and 64 lanes (the larger capacities) first combine across rows
// with lane shuffles (symmetric, so the lanes still agree bit for bit).
__device__ __forceinline__ double group_sum_wide(double v, int G) {
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  return group_sum(v, G);
}

// The same butterfly for V independent values at once with a compile-time
// group size 2^LG, so the steps of the V values interleave; the runtime
// form branches once on the (wave-uniform) group size.  Wide adds the
// cross-row steps for groups of 32 and 64 lanes.
template <int LG, int V>
__device__ __forceinline__ void group_sum_fixed(double (&v)[V]) {
  if constexpr (LG >= 6) {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] += __shfl_xor(v[i], 32, 64);
  }
  if constexpr (LG >= 5) {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] += __shfl_xor(v[i], 16, 64);
  }
  if constexpr (LG >= 4) {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] += dpp_d<kDppMirror>(v[i]);
  }
  if constexpr (LG >= 3) {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] += dpp_d<kDppHalfMirror>(v[i]);
  }
  if constexpr (LG >= 1) {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] += dpp_d<kDppXor1>(v[i]);
  }
  if constexpr (LG >= 2) {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] += dpp_d<kDppXor2>(v[i]);
  }
}
template <bool Wide, int V>
__device__ __forceinline__ void group_sum_n(double (&v)[V], int G) {
  switch (G) {
    case 1: break;
    case 2: group_sum_fixed<1>(v); break;
    case 4: group_sum_fixed<2>(v); break;
    case 8: group_sum_fixed<3>(v); break;
    case 16: group_sum_fixed<4>(v); break;
    default:
      if constexpr (Wide) {
        if (G == 32)
          group_sum_fixed<5>(v);
        else
          group_sum_fixed<6>(v);
      }
      break;
  }
}

// idx = start, start + step, ... split as idx = q W + r without a division
// per element (an integer division by a runtime divisor costs tens of
// instructions on this ISA): the quotient and remainder advance by those of
// the step.
struct DivWalk {
  int idx, q, r;
  int step, dq, dr, W;
  __device__ __forceinline__ DivWalk(int start, int step_, int W_)
      : idx(start), q(start / W_), r(start - (start / W_) * W_), step(step_), dq(step_ / W_),
        dr(step_ - (step_ / W_) * W_), W(W_) {}
  __device__ __forceinline__ void next() {
    idx += step;
    q += dq;
    r += dr;
    if (r >= W) {
      r -= W;
      ++q;
    }
  }
};

// Reciprocal square root and reciprocal from the hardware estimate refined by
// one Newton step (the estimate's relative error is squared away), so the
// rotation parameters cost two short dependent chains instead of the IEEE
// sqrt/divide sequences.
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// Lanes per group so that n groups fit in NT lanes, at most 16.
__device__ __forceinline__ int lanes_per(int n, int NT) {
  int g = 1;
  while (g < 16 && n * g * 2 <= NT) g <<= 1;
  return g;
}

// Wave-uniform helpers built on DPP row operations and readlane.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffu), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, true);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}
// Max over the 64 lanes of a wave (all lanes active); wave-uniform result.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
  k = umax64(k, dpp_u64<kDppMirror>(k));
  k = umax64(k, dpp_u64<kDppHalfMirror>(k));
  k = umax64(k, dpp_u64<kDppXor1>(k));
  k = umax64(k, dpp_u64<kDppXor2>(k));
  unsigned long long m = 0;
  for (int r = 0; r < 4; ++r) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(k & 0xffffffffu), 16 * r);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(k >> 32), 16 * r);
    m = umax64(m, ((unsigned long long)hi << 32) | lo);
  }
  return m;
}
// Sum over the 64 lanes of a wave in a fixed order; wave-uniform result.
__device__ __forceinline__ double wave_sum(double v) {
  v = group_sum(v, 16);
  return ((readlane_d(v, 0) + readlane_d(v, 16)) + readlane_d(v, 32)) + readlane_d(v, 48);
}
// Argmax key of a non-negative value at index c < 256: larger values win,
// ties (to 2^-44 relative) go to the smaller index.
__device__ __forceinline__ unsigned long long argmax_key(double v, int c) {
  if (!(v >= 0.0)) return 0ull;
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b & ~255ull) | (unsigned long long)(255 - c);
}
__device__ __forceinline__ int argmax_index(unsigned long long key) {
  return 255 - (int)(key & 255ull);
}

// ----------------------------------------------------------------------------
// Row blocks.  A column of n rows is padded with zero rows to a power of two
// `pad` and split over G lanes, lane q owning the contiguous rows
// q*RPL .. q*RPL+RPL-1 (RPL = pad / G, a compile-time constant of the inner
// loops, so they are straight-line code with immediate LDS offsets).
__device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }


}  // namespace tnrg
