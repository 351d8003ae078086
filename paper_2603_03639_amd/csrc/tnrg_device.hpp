// Device building blocks of the MPS robust-GRAPE hot path for gfx950 that
// touch the per-workgroup working buffers.
//
// One workgroup owns one trajectory (one crosstalk sample k and one input r).
// Everything a bond update touches -- the two site tensors, the two-site
// matrix theta and the one-sided Jacobi working copy -- lives in one set of
// working buffers.  The MPS itself lives in HBM in a fixed-capacity layout
// (include/tnrg.h) and is streamed site by site during a sweep, so a slice
// reads and writes every site once.
//
// This file is included once per memory space of the working buffers:
// TNRG_NS names the namespace and TNRG_AS qualifies the buffer pointers.
// With TNRG_AS = address_space(3) the buffers are LDS and every access
// compiles to ds_read / ds_write (capacities up to 32); with TNRG_AS empty
// they are per-workgroup global scratch reached through flat pointers (the
// larger capacities, whose working set exceeds the 160 KB of LDS).
#include "tnrg_common.hpp"

#if !defined(TNRG_NS) || !defined(TNRG_AS) || !defined(TNRG_BIG)
#error "define TNRG_NS, TNRG_AS and TNRG_BIG before including tnrg_device.hpp"
#endif

namespace TNRG_NS {

using namespace tnrg;

typedef TNRG_AS c2 sc2;
typedef TNRG_AS double sdbl;
typedef TNRG_AS int sint;
typedef TNRG_AS long long sll;

// The LDS variant serves capacities up to 32: bond problems of at most 64
// columns (one value per lane in the wave-level pivot search and sort), lane
// groups of at most 16 and, by the launch configuration, all column pairs of
// a Jacobi round at once.  The global-scratch variant serves up to 256
// columns (four values per lane), groups of up to 64 lanes and rounds with
// more pairs than lane groups.
constexpr bool kWide = TNRG_BIG;
// Depth steps of 4 whose operands a matrix-core product tile loads at once:
// 4 in the global-scratch build, whose operands come from L2 and whose depths
// reach 256; 1 in the LDS build, whose depths of at most 64 (mostly 16) come
// from LDS (measured at bond dimension 16: batching 8 steps cost 1 % there).
constexpr int kMfmaSteps = TNRG_BIG ? 4 : 1;
constexpr int kLaneQuads = TNRG_BIG ? 4 : 1;
__device__ __forceinline__ double gsum(double v, int G) {
  double red[1] = {v};
  group_sum_n<kWide>(red, G);
  return red[0];
}

typedef TNRG_AS Layout sLayout;
__device__ __forceinline__ void layout_build(sLayout& L, int N, int dcap) {
  if (threadIdx.x == 0) {
    L.N = N;
    L.dcap = dcap;
    long long o = 0;
    for (int b = 0; b <= N; ++b) L.cap[b] = bond_cap(N, dcap, b);
    for (int j = 0; j < N; ++j) {
      L.off[j] = o;
      o += (long long)L.cap[j] * 2 * L.cap[j + 1];
    }
    L.off[N] = o;
  }
  __syncthreads();
}

// Per-workgroup context.  LDS buffers are sized from P2 = max(4, pow2(2 cap)):
//   LC, LO : P2^2 / 2 complex each (centre tensor, other tensor / isometry Q;
//            together the LQ working matrix)
//   X      : P2 (P2 + 1) complex (Jacobi working matrix)
//   sig    : P2 doubles, perm : P2 ints
struct Ctx {
  int tid, nt;
  int cap;
  sc2* LC;
  sc2* LO;
  sc2* X;
  sdbl* sig;
  sint* perm;
  c2* X0;       // global scratch (P2 (P2 + 1)), the unrotated theta
  sLayout* L;   // layout of the internal states
  sint* sdims;  // LDS [kMaxSites + 1]
  ModelDev md;
  // per-trajectory bookkeeping in LDS (written by thread 0)
  sint* sflag;
  // [kStats]: max dim, max sweeps, total sweeps, svd count, Jacobi flops,
  // contraction flops (theta, projection, environments), Jacobi rounds, LQ
  // steps, then phase
  // clock ticks: site load/store, theta, LQ, Jacobi, split finish, left
  // environments, right environments + insertions, whole kernel.
  sll* sstat;
  sdbl* red;       // LDS [kMaxWaves * 8]
  sint* sk;          // LDS scalar: kept singular values of the last split
  sdbl* sinv;        // LDS scalar: 1 / norm of kept singular values
  sdbl* sd;          // LDS scratch scalars [4]
  sint* si;          // LDS scratch scalars [4]
  // global-scratch build: dynamic LDS that holds the Jacobi matrix of a bond
  // update when it fits (jx_elems complex, 0 when there is none)
  __attribute__((address_space(3))) c2* jx;
  int jx_elems;
};

__device__ __forceinline__ void flag_or(Ctx& C, int v) {
  __hip_atomic_fetch_or(C.sflag, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Phase timer (thread 0, constant-rate wall clock), active when md.profile.
__device__ __forceinline__ long long ph_now(const Ctx& C) {
  return (C.md.profile && C.tid == 0) ? (long long)wall_clock64() : 0;
}
__device__ __forceinline__ void ph_add(Ctx& C, int slot, long long& t0) {
  if (C.md.profile && C.tid == 0) {
    const long long t1 = (long long)wall_clock64();
    C.sstat[slot] += t1 - t0;
    t0 = t1;
  }
}

// ----------------------------------------------------------------------------
// Block-wide deterministic reduction of V complex values (V <= 4).  Every
// thread passes its partial sums; the result is returned to every thread.
// The summation order is fixed (butterfly inside each wave, waves in order).
template <int V>
__device__ __forceinline__ void block_sum(Ctx& C, c2 (&v)[V]) {
  for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      v[i].x += __shfl_xor(v[i].x, o, 64);
      v[i].y += __shfl_xor(v[i].y, o, 64);
    }
  }
  const int w = C.tid >> 6, nw = (C.nt + 63) >> 6;
  if ((C.tid & 63) == 0) {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      C.red[w * 8 + 2 * i] = v[i].x;
      C.red[w * 8 + 2 * i + 1] = v[i].y;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < V; ++i) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < nw; ++k) {
      sr += C.red[k * 8 + 2 * i];
      si += C.red[k * 8 + 2 * i + 1];
    }
    v[i] = cmk(sr, si);
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// Pivoted Householder LQ (QR with column pivoting of X^dag) as the
// preconditioner of the one-sided Jacobi SVD.  Z (column-major, column r at
// Z + r*ldz, ldz = pad(nz) rows with zero padding) holds X^dag: column r of Z
// is the conjugated row r of X.  On return the lower-trapezoidal
// L = P R^dag (len x rank, len = mz) with X = L Q^dag, Q orthonormal, is
// written column-major into X (ldx, rows padded with zeros to pad(mz)); L has
// the singular values and left singular vectors of X.  Columns of Z whose
// remaining norm falls to thr2 = (len eps)^2 ||X||_F^2 stop the factorisation
// (numerical rank).  Returns the rank (>= 1).  mz <= 256.
// Scratch: nrm = C.sig (remaining squared norms by logical column), pcol =
// C.perm (logical -> physical column of Z).
// Per-lane register copies of a small table indexed by position c < 64 *
// kLaneQuads: lane l holds the entries l, l + 64, ...  Every wave keeps its
// own copy, updated identically, so the table needs no LDS or barrier.
template <class T>
__device__ __forceinline__ T quad_pick(const T (&r)[kLaneQuads], int q) {
  T v = r[0];
#pragma unroll
  for (int i = 1; i < kLaneQuads; ++i) v = (q == i) ? r[i] : v;
  return v;
}
// entry c (wave-uniform c)
__device__ __forceinline__ int table_at(const int (&r)[kLaneQuads], int c) {
  return __builtin_amdgcn_readlane(quad_pick(r, c >> 6), c & 63);
}
__device__ __forceinline__ double table_at(const double (&r)[kLaneQuads], int c) {
  return readlane_d(quad_pick(r, c >> 6), c & 63);
}
// entry c (c per lane, 0 <= c < 64 kLaneQuads)
__device__ __forceinline__ int table_gather(const int (&r)[kLaneQuads], int c) {
  int out = 0;
#pragma unroll
  for (int i = 0; i < kLaneQuads; ++i) {
    const int t = __shfl(r[i], c & 63, 64);
    out = ((c >> 6) == i) ? t : out;
  }
  return out;
}

template <int RQ>
__device__ __forceinline__ void lq_apply(Ctx& C, sc2* Z, int ldz, int j, int mz, int G, const sc2* zp, c2 v0,
                         double coef, sdbl* nrm_next, const int (&pcol)[kLaneQuads], int best,
                         int pj) {
  const int tid = C.tid, NT = C.nt;
  const int grp = tid / G, q = tid % G;
  const int ngrp = NT / G;
  const int r0 = q * RQ;
  // v_i = 0 (i < j), v0 (i = j), zp_i (i > j)
  c2 v[RQ];
#pragma unroll
  for (int i = 0; i < RQ; ++i) {
    const int row = r0 + i;
    const c2 z = zp[row];
    v[i] = row < j ? cmk(0.0, 0.0) : (row == j ? v0 : z);
  }
  const int ncols = mz - j - 1;
  // the trip count is the same for every lane (the column map gather is a
  // lane shuffle); groups past the last column work on nothing
  for (int c0 = 0; c0 < ncols; c0 += ngrp) {
    const int c = j + 1 + c0 + grp;
    const bool live = c0 + grp < ncols;
    // this step's pivot swap applies here: position best now holds the
    // column that was at position j
    const int phys = table_gather(pcol, live ? c : 0);
    if (!live) continue;
    sc2* zc = Z + (c == best ? pj : phys) * ldz + r0;
    c2 z[RQ];
#pragma unroll
    for (int i = 0; i < RQ; ++i) z[i] = zc[i];
    c2 w = cmk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < RQ; ++i) w = cfmac(v[i], z[i], w);
    {
      double red[2] = {w.x, w.y};
      group_sum_n<kWide>(red, G);
      w = cmk(red[0], red[1]);
    }
    const c2 cw = cscale(w, coef);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < RQ; ++i) {
      z[i] = csub(z[i], cmul(v[i], cw));
      zc[i] = z[i];
      if (r0 + i > j) s += cabs2(z[i]);
    }
    s = gsum(s, G);
    if (q == 0) nrm_next[c] = s;
  }
}

// The pivot search of a step runs in every wave on the same LDS values, so
// the pivot, the Householder scalars and the stop decision are wave-uniform
// registers everywhere and need no broadcast; the column map lives in
// registers of every wave (updated identically) and the remaining column
// norms are double buffered (read from one LDS buffer, the updated ones
// written to the other), so a step needs a single barrier.  The R diagonal
// of a step is written into Z at the start of the next step, when no wave
// reads that element any more.
__device__ __forceinline__ int lq_pivot(Ctx& C, sc2* Z, int nz, int mz, int ldz, sc2* X, int ldx, double* thr2_out) {
  const int tid = C.tid, NT = C.nt;
  const int lane = tid & 63;
  sdbl* nrm = C.sig;
  sdbl* nrm2 = (sdbl*)X;  // X is free until L is written into it
  const int padz = ldz;
  const int G = uniform(max(min(lanes_per(mz, NT), padz), padz / 8));
  const int RQ = uniform(padz / G);
  {
    const int grp = tid / G, q = tid % G;
    for (int c = grp; c < mz; c += NT / G) {
      double s = 0.0;
      for (int i = 0; i < RQ; ++i) s += cabs2(Z[c * ldz + q * RQ + i]);
      s = gsum(s, G);
      if (q == 0) nrm[c] = s;
    }
  }
  int pcol[kLaneQuads];
#pragma unroll
  for (int q = 0; q < kLaneQuads; ++q) pcol[q] = lane + 64 * q;
  __syncthreads();
  // threshold (len eps)^2 ||X||_F^2, computed by every wave
  double thr2;
  {
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kLaneQuads; ++q) {
      const int c = lane + 64 * q;
      part += c < mz ? nrm[c] : 0.0;
    }
    const double f2 = wave_sum(part);
    const double lt = (double)mz * 2.220446049250313e-16;
    thr2 = lt * lt * f2;
  }
  *thr2_out = thr2;
  const int steps = nz < mz ? nz : mz;
  int rank = steps;
  int pend_col = -1, pend_row = 0;
  c2 pend_val = cmk(0.0, 0.0);
  sdbl* cur = nrm;
  sdbl* nxt = nrm2;
  for (int j = 0; j < steps; ++j) {
    if (tid == 0 && pend_col >= 0) Z[pend_col * ldz + pend_row] = pend_val;
    double nv[kLaneQuads];
    unsigned long long kk = 0ull;
#pragma unroll
    for (int q = 0; q < kLaneQuads; ++q) {
      const int c = lane + 64 * q;
      nv[q] = (c >= j && c < mz) ? cur[c] : 0.0;
      kk = umax64(kk, (c >= j && c < mz) ? argmax_key(nv[q], c) : 0ull);
    }
    const unsigned long long key = wave_max_u64(kk);
    const int best = argmax_index(key);
    const double bv = table_at(nv, best);
    if (!(key != 0ull && bv > thr2)) {
      rank = j;
      break;
    }
    if (tid == 0) C.sstat[7] += 1;  // LQ steps
    const int pj = table_at(pcol, j);
    const int pb = table_at(pcol, best);
    const sc2* zp = Z + pb * ldz;
    const c2 x0 = zp[j];
    const double xn = bv * rsqrt_nr(bv);
    const double a2 = cabs2(x0);
    const double rax = a2 > 0.0 ? rsqrt_nr(a2) : 0.0;
    const double ax0 = a2 * rax;
    const c2 ph = a2 > 0.0 ? cscale(x0, rax) : cmk(1.0, 0.0);
    // v = x + ph ||x|| e_j,  H x = -ph ||x|| e_j,  H = I - coef v v^dag
    const c2 v0 = cmk(x0.x + ph.x * xn, x0.y + ph.y * xn);
    const double coef = rcp_nr(xn * (xn + ax0));
    switch (RQ) {
      case 1: lq_apply<1>(C, Z, ldz, j, mz, G, zp, v0, coef, nxt, pcol, best, pj); break;
      case 2: lq_apply<2>(C, Z, ldz, j, mz, G, zp, v0, coef, nxt, pcol, best, pj); break;
      case 4: lq_apply<4>(C, Z, ldz, j, mz, G, zp, v0, coef, nxt, pcol, best, pj); break;
      default: lq_apply<8>(C, Z, ldz, j, mz, G, zp, v0, coef, nxt, pcol, best, pj); break;
    }
    // the swap in the column map
#pragma unroll
    for (int q = 0; q < kLaneQuads; ++q) {
      const int c = lane + 64 * q;
      pcol[q] = (c == j) ? pb : ((c == best) ? pj : pcol[q]);
    }
    pend_col = pb;
    pend_row = j;
    pend_val = cmk(-ph.x * xn, -ph.y * xn);
    sdbl* t = cur;
    cur = nxt;
    nxt = t;
    __syncthreads();
  }
  if (tid == 0 && pend_col >= 0) Z[pend_col * ldz + pend_row] = pend_val;
  if (tid < 64) {
#pragma unroll
    for (int q = 0; q < kLaneQuads; ++q)
      if (lane + 64 * q < mz) C.perm[lane + 64 * q] = pcol[q];
  }
  __syncthreads();
  sint* pcolm = C.perm;
  if (rank < 1) rank = 1;  // a zero matrix still yields one (zero) column
  // L[pcol[c]][i] = conj(R[i][c]) = conj(Z[pcol[c]][i]) for i <= c, 0 below;
  // padding rows mz .. pad-1 of every column are zero.
  const int padx = pow2_at_least(mz);
  for (DivWalk w(tid, NT, padx); w.idx < rank * padx; w.next()) {
    const int i = w.q, c = w.r;
    c2 val = cmk(0.0, 0.0);
    int row = c;
    if (c < mz) {
      row = pcolm[c];
      if (i <= c) val = cconj(Z[row * ldz + i]);
    }
    X[i * ldx + row] = val;
  }
  __syncthreads();
  return rank;
}

// ----------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of the len x ncol matrix X held column-major
// in LDS (column c at X + c*ldx, rows padded with zeros to pad = pow2(len)).
// Columns are rotated pairwise until every pair is orthogonal to len * 2^-52
// relative to the column norms (a sweep whose rotations all had
// |sin|^2 < 2^-52 ends the iteration: the cosines it leaves are at most about
// n 2^-52 <= len 2^-52, so the next sweep would rotate nothing); the
// columns then hold sigma_i u_i.  Pairs
// are visited in the round-robin (circle) order, all disjoint pairs of a
// round in parallel; each pair's rows are split over G lanes whose partial
// dot products are combined by a DPP butterfly, so every lane of the pair
// derives the same rotation.  Columns whose squared norm is at most thr2
// (rounding level of the whole matrix) take no part in rotations; after each
// sweep they are dropped and the live columns are packed to the front, in
// order.  Returns the number of live columns (>= 1); sig[c] holds ||X_c|| for
// those.  *sweeps_out receives the number of sweeps.
template <int RPL, class T>
__device__ __forceinline__ int jacobi_sweep(Ctx& C, T* X, int ldx, int n, int G, double thr2,
                                            double tol2, T* dummy) {
  const int tid = C.tid;
  const int P = (n + 1) >> 1;
  const int m = 2 * P - 1;
  const int grp = tid / G, q = tid % G;
  const int ngrp = C.nt / G;
  const int r0 = q * RPL;
  int rotated = 0;  // bit 0: a rotation; bit 1: a rotation with |sin|^2 >= 2^-52
  // one pair (ia, ib) of one round; idle slots work on two scratch columns
  // nobody reads, so the round is straight-line code without lane masking
  auto pair = [&](int ia, int ib, bool valid) {
    T* xc = (valid ? X + ia * ldx : dummy) + r0;
    T* yc = (valid ? X + ib * ldx : dummy + G * RPL) + r0;
    c2 x[RPL], y[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      x[i] = xc[i];
      y[i] = yc[i];
    }
    double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      a = fma(x[i].x, x[i].x, fma(x[i].y, x[i].y, a));
      b = fma(y[i].x, y[i].x, fma(y[i].y, y[i].y, b));
      gr = fma(x[i].x, y[i].x, fma(x[i].y, y[i].y, gr));
      gi = fma(x[i].x, y[i].y, fma(-x[i].y, y[i].x, gi));
    }
    {
      double red[4] = {a, b, gr, gi};
      group_sum_n<kWide>(red, G);
      a = red[0];
      b = red[1];
      gr = red[2];
      gi = red[3];
    }
    const double g2 = fma(gr, gr, gi * gi);
    const bool rot = valid && a > thr2 && b > thr2 && g2 > tol2 * a * b;
    rotated |= rot ? 1 : 0;
    // With d = b - a, h = sqrt(d^2 + 4|gamma|^2) and u = |d| + h the
    // rotation that zeroes the pair's inner product has
    //   tan(theta) e = 2 sgn(d) gamma / u,   c = u w,   s e = 2 sgn(d) w gamma,
    // w = 1/sqrt(u^2 + 4|gamma|^2) = 1/sqrt(2 h u) = (1/h) / sqrt(2 (1 + |d|/h)).
    // A pair that is not rotated gets the identity (c = 1, s = 0).
    const double d = b - a;
    const double s2 = fma(d, d, 4.0 * g2);
    const double rh = rsqrt_nr(s2);
    const double ad = fabs(d);
    const double w = rh * rsqrt_nr(2.0 * fma(ad, rh, 1.0));
    const double cs = rot ? fma(s2, rh, ad) * w : 1.0;
    const double sw2 = rot ? (d >= 0.0 ? 2.0 : -2.0) * w : 0.0;
    const double pr = sw2 * gr, pi = sw2 * gi;  // s e
    rotated |= (rot && sw2 * sw2 * g2 >= 2.220446049250313e-16) ? 2 : 0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      c2 xn, yn;
      // x' = c x - conj(s e) y,  y' = (s e) x + c y
      xn.x = cs * x[i].x - (pr * y[i].x + pi * y[i].y);
      xn.y = cs * x[i].y - (pr * y[i].y - pi * y[i].x);
      yn.x = cs * y[i].x + (pr * x[i].x - pi * x[i].y);
      yn.y = cs * y[i].y + (pr * x[i].y + pi * x[i].x);
      xc[i] = xn;
      yc[i] = yn;
    }
    if (valid && !(a == a && b == b && g2 == g2)) flag_or(C, 4);
  };
  // Round r of the circle schedule pairs column 0 with column 1 + r and,
  // for slot p = 1 .. P-1, column 1 + (p + r) mod m with 1 + (m - p + r) mod m.
  if (!kWide || P <= ngrp) {
    // one slot per lane group: the positions advance by one each round
    const int pp = grp;
    int ia = (pp == 0) ? 0 : 1 + pp;
    int ib = (pp == 0) ? 1 : 1 + m - pp;
    const bool slot_ok = pp < P;
    for (int r = 0; r < m; ++r) {
      pair(ia, ib, slot_ok && ia < n && ib < n);
      if (pp == 0) {
        ib = (ib == m) ? 1 : ib + 1;
      } else {
        ia = (ia == m) ? 1 : ia + 1;
        ib = (ib == m) ? 1 : ib + 1;
      }
      __syncthreads();
    }
  } else {
    // more pairs than lane groups: every group takes the slots grp,
    // grp + ngrp, ... of each round in turn (the pairs of a round are
    // disjoint, so their order does not matter)
    const int nslot = (P + ngrp - 1) / ngrp;
    for (int r = 0; r < m; ++r) {
      for (int u = 0; u < nslot; ++u) {
        const int pp = grp + u * ngrp;
        const int ia = (pp == 0) ? 0 : 1 + (pp + r) % m;
        const int ib = (pp == 0) ? 1 + r : 1 + (m - pp + r) % m;
        pair(ia, ib, pp < P && ia < n && ib < n);
      }
      __syncthreads();
    }
  }
  return rotated;
}

// X and dummy (two scratch columns of pad rows for idle pair slots) are in
// LDS or in global scratch (T is the element type with its address space).
template <class T>
__device__ __forceinline__ int jacobi_lds(Ctx& C, T* X, int len, int ncol, int ldx, double thr2,
                                          int* sweeps_out, T* dummy) {
  const int tid = C.tid, NT = C.nt;
  const double tol = (double)len * 2.220446049250313e-16;
  const double tol2 = tol * tol;
  const int pad = pow2_at_least(len);
  int n = ncol;
  int sweeps = 0;
  const int max_sweeps = C.md.max_sweeps;
  // column norms of the first n columns into sig (squared)
  auto norms = [&](int nn) {
    const int Gc = min(lanes_per(nn, 2 * NT), pad);
    const int Rc = pad / Gc;
    const int gc = tid / Gc, qc = tid % Gc;
    for (int c = gc; c < nn; c += NT / Gc) {
      const T* xc = X + c * ldx + qc * Rc;
      double s = 0.0;
      for (int i = 0; i < Rc; ++i) s += cabs2(xc[i]);
      double red[1] = {s};
      group_sum_n<kWide>(red, Gc);
      if (qc == 0) C.sig[c] = red[0];
    }
  };
  for (int sw = 0; sw < max_sweeps && n >= 2; ++sw) {
    const int P = (n + 1) >> 1;
    // at most 8 rows per lane (groups of up to 32 lanes for 256 rows)
    const int G = uniform(max(min(lanes_per(P, NT), pad), pad / 8));
    int rotated;
    long long tj = ph_now(C);
    switch (uniform(pad / G)) {
      case 1: rotated = jacobi_sweep<1>(C, X, ldx, n, G, thr2, tol2, dummy); break;
      case 2: rotated = jacobi_sweep<2>(C, X, ldx, n, G, thr2, tol2, dummy); break;
      case 4: rotated = jacobi_sweep<4>(C, X, ldx, n, G, thr2, tol2, dummy); break;
      default: rotated = jacobi_sweep<8>(C, X, ldx, n, G, thr2, tol2, dummy); break;
    }
    ++sweeps;
    if (tid == 0) {
      C.sstat[4] += 18LL * len * n * (n - 1);
      C.sstat[6] += 2 * P - 1;  // rounds
    }
    ph_add(C, kPhJacRounds, tj);
    const int any = __syncthreads_or(rotated & 1);
    // Quadratic convergence: a sweep whose rotations all had |sin|^2 < 2^-52
    // leaves cosines of at most about n 2^-52, within the tolerance len 2^-52,
    // so the confirming sweep without rotations is skipped.
    const int anybig = __syncthreads_or(rotated & 2);
    if (sw == 0 && any) {
      // after the first sweep, drop the columns that sank to rounding level
      // and pack the live ones to the front in order
      norms(n);
      __syncthreads();
      // new positions by a prefix count of the live columns (every wave
      // computes it; wave 0 writes the map)
      int nn = 0;
#pragma unroll
      for (int q = 0; q < kLaneQuads; ++q) {
        const int c = (tid & 63) + 64 * q;
        const bool live = c < n && C.sig[c] > thr2;
        const unsigned long long ball = __ballot(live);
        const int before = __popcll(ball & ((1ull << (tid & 63)) - 1ull));
        if (tid < 64 && c < n) C.perm[c] = live ? nn + before : -1;
        nn += __popcll(ball);
      }
      __syncthreads();
      if (nn < n) {
        // move live column c to position perm[c] (<= c) in increasing order
        // of c, so no source is overwritten before it is read
        for (int c = 0; c < n; ++c) {
          const int dst = C.perm[c];
          if (dst >= 0 && dst != c) {
            for (int row = tid; row < pad; row += NT) X[dst * ldx + row] = X[c * ldx + row];
            __syncthreads();
          }
        }
        n = nn > 0 ? nn : 1;
      }
    }
    ph_add(C, kPhJacSweepEnd, tj);
    if (!any || !anybig) break;
    if (sw + 1 == max_sweeps) {
      if (tid == 0) flag_or(C, 2);
      break;
    }
  }
  norms(n);
  __syncthreads();
  for (int c = tid; c < n; c += NT) C.sig[c] = sqrt(C.sig[c]);
  __syncthreads();
  *sweeps_out = sweeps;
  return n;
}

// Sort the n singular values (descending, ties by column index), choose the
// kept count k by the truncation rule and compute 1/||sigma_{1..k}||.
// n <= 256 (one wave decides, up to four values per lane).
__device__ __forceinline__ void choose_k(Ctx& C, int n, int len, int capk) {
  if (C.tid < 64) {
    const int lane = C.tid;
    double v[kLaneQuads];
    int rk[kLaneQuads];
    unsigned long long kk = 0ull;
#pragma unroll
    for (int q = 0; q < kLaneQuads; ++q) {
      v[q] = -1.0;
      rk[q] = 0;
      if (q * 64 < n) {
        const int c = lane + 64 * q;
        double x = (c < n) ? C.sig[c] : -1.0;
        if (!(x == x)) x = -1.0;
        int rank = 0;
#pragma unroll 4
        for (int d = 0; d < n; ++d) {
          double w = C.sig[d];
          if (!(w == w)) w = -1.0;
          rank += (w > x) || (w == x && d < c);
        }
        if (c < n) {
          C.perm[rank] = c;
          kk = umax64(kk, argmax_key(x, c));
        }
        v[q] = x;
        rk[q] = rank;
      }
    }
    const unsigned long long key = wave_max_u64(kk);
    const double smax = (key != 0ull) ? C.sig[argmax_index(key)] : 0.0;
    int k = 0;
#pragma unroll
    for (int q = 0; q < kLaneQuads; ++q)
      if (q * 64 < n) k += __popcll(__ballot(lane + 64 * q < n && v[q] >= C.md.eps * smax));
    if (k > C.md.chi) k = C.md.chi;
    if (k < 1) k = 1;
    const int lim = len < n ? len : n;
    if (k > lim) k = lim;
    int over = 0;
    if (k > capk) {
      over = 1;
      k = capk;
    }
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kLaneQuads; ++q)
      if (lane + 64 * q < n && rk[q] < k) part += v[q] * v[q];
    const double s2 = wave_sum(part);
    if (lane == 0) {
      if (over) flag_or(C, 1);
      if (!(smax > 0.0) || !(s2 == s2)) flag_or(C, 4);
      C.sk[0] = k;
      C.sinv[0] = (C.md.renorm && s2 > 0.0) ? 1.0 / sqrt(s2) : 1.0;
      if (k > C.sstat[0]) C.sstat[0] = k;
    }
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// Site tensor transfer between HBM (capacity layout) and LDS (packed), with a
// single-site 2x2 gate applied on the physical index: out[a,s,c] = sum_t
// G[s][t] in[a,t,c].
__device__ __forceinline__ void load_site(Ctx& C, sc2* dst, const c2* site, int dl, int dr, int capr,
                          const M22& G) {
  const int n = dl * 2 * dr;
  for (DivWalk w(C.tid, C.nt, 2 * dr); w.idx < n; w.next()) {
    const int a = w.q;
    const int s = w.r >= dr ? 1 : 0;
    const int c = w.r - s * dr;
    const c2 x0 = site[(size_t)(a * 2 + 0) * capr + c];
    const c2 x1 = site[(size_t)(a * 2 + 1) * capr + c];
    dst[w.idx] = m22_row(G, s, x0, x1);
  }
}
__device__ __forceinline__ void store_site(Ctx& C, c2* site, const sc2* src, int dl, int dr, int capr,
                           const M22& G) {
  const int n = dl * 2 * dr;
  for (DivWalk w(C.tid, C.nt, 2 * dr); w.idx < n; w.next()) {
    const int a = w.q;
    const int s = w.r >= dr ? 1 : 0;
    const int c = w.r - s * dr;
    const c2 x0 = src[(a * 2 + 0) * dr + c];
    const c2 x1 = src[(a * 2 + 1) * dr + c];
    site[(size_t)(a * 2 + s) * capr + c] = m22_row(G, s, x0, x1);
  }
}

// ----------------------------------------------------------------------------
// Two-site update of one bond (Sec. II: apply the two-qubit gate, split by an
// SVD, compress).  Lt (dl,2,dm) and Rt (dm,2,dr) are packed in LDS; the gate
// bg is the bond exponential (the ZZ phase, or the Heisenberg bond gate).
//   ltr: left factor U (left-isometric) is written to `iso` (site b, capacity
//        row stride iso_capr) after the gate Gfin, the centre diag(s) V^dag
//        (k,2,dr) is left in LC.
//   rtl: right factor V^dag is written to `iso` (site b+1), the centre
//        U diag(s) (dl,2,k) is left in LC.
// iso may be null (nothing written).  Returns k, the new bond dimension.
__device__ __forceinline__ int bond_split(Ctx& C, const sc2* Lt, const sc2* Rt, int dl, int dm, int dr,
                          const BondGate& bg, bool ltr, c2* iso, int iso_capr, const M22& Gfin,
                          int capk) {
  long long t0 = ph_now(C);
  const int len = ltr ? 2 * dl : 2 * dr;
  const int nc = ltr ? 2 * dr : 2 * dl;
  const int ldx = pow2_at_least(len) + 1;
  sc2* X = C.X;
  c2* X0 = C.X0;
  const bool offd = C.md.heis;
  // theta[(a,s),(s',c)] = sum_b Lt[a,s,b] Rt[b,s',c], then the gate, which
  // couples (s,s') only with (1-s,1-s'): one item makes the pair
  // (0,s') / (1,1-s') of row pair a and column c
  const int npair = 2 * dl * dr;
  if (!offd && dm > 32) {
    // large inner bond (global-scratch build only, so both builds agree
    // bitwise on every problem they share): theta on the matrix cores, the
    // diagonal bond gate (phase index s xor s') applied as each element is
    // stored
    cgemm_mfma<kMfmaSteps>(
        C.tid, C.nt, 2 * dl, 2 * dr, dm,
        [&](int r, int b) { return Lt[r * dm + b]; },
        [&](int b, int col) { return Rt[b * 2 * dr + col]; },
        [&](int r, int col, c2 t) {
          const int sx = (r & 1) ^ (col >= dr ? 1 : 0);
          const c2 v = cmul(t, sx ? bg.d[1] : bg.d[0]);
          if (ltr) {
            X[col * ldx + r] = v;
            X0[col * ldx + r] = v;
          } else {
            X[r * ldx + col] = cconj(v);
            X0[r * ldx + col] = cconj(v);
          }
        });
  } else
  for (DivWalk w(C.tid, C.nt, 2 * dr); w.idx < npair; w.next()) {
    const int a = w.q;
    const int col0 = w.r;
    const int s2 = col0 >= dr ? 1 : 0;
    const int c = col0 - s2 * dr;
    const int col1 = col0 + (s2 ? -dr : dr);
    const int row0 = 2 * a, row1 = 2 * a + 1;
    const sc2* lp0 = Lt + row0 * dm;
    const sc2* lp1 = Lt + row1 * dm;
    const sc2* rp0 = Rt + s2 * dr + c;
    const sc2* rp1 = Rt + (1 - s2) * dr + c;
    c2 t0v = cmk(0.0, 0.0), t1v = cmk(0.0, 0.0);
#pragma unroll 4
    for (int b = 0; b < dm; ++b) {
      t0v = cfma(lp0[b], rp0[b * 2 * dr], t0v);
      t1v = cfma(lp1[b], rp1[b * 2 * dr], t1v);
    }
    const c2 d = s2 ? bg.d[1] : bg.d[0];
    c2 v0 = cmul(t0v, d), v1 = cmul(t1v, d);
    if (offd) {
      const c2 o = s2 ? bg.o[1] : bg.o[0];
      v0 = cfma(o, t1v, v0);
      v1 = cfma(o, t0v, v1);
    }
    if (ltr) {
      X[col0 * ldx + row0] = v0;
      X0[col0 * ldx + row0] = v0;
      X[col1 * ldx + row1] = v1;
      X0[col1 * ldx + row1] = v1;
    } else {
      X[row0 * ldx + col0] = cconj(v0);
      X0[row0 * ldx + col0] = cconj(v0);
      X[row1 * ldx + col1] = cconj(v1);
      X0[row1 * ldx + col1] = cconj(v1);
    }
  }
  __syncthreads();
  // Z = X^dag (nc x len, rows padded to pow2(nc)) in LC..LO, pivoted LQ ->
  // L (len x rank) in X
  sc2* Z = C.LC;
  const int ldz = pow2_at_least(nc);
  for (DivWalk w(C.tid, C.nt, ldz); w.idx < len * ldz; w.next()) {
    const int r = w.q, c = w.r;
    Z[w.idx] = c < nc ? cconj(X[c * ldx + r]) : cmk(0.0, 0.0);
  }
  __syncthreads();
  ph_add(C, kPhTheta, t0);
  double thr2;
  const int rank = lq_pivot(C, Z, nc, len, ldz, X, ldx, &thr2);
  ph_add(C, kPhLQ, t0);
  int sw = 0;
  int nlive;
  const int padl = pow2_at_least(len);
  if (TNRG_BIG && (long long)rank * ldx + 2 * padl <= C.jx_elems) {
    // global-scratch build: the Jacobi runs on an LDS copy of L (the idle
    // pair slots' scratch columns after it), which goes back for the finish
    auto* J = C.jx;
    for (int i = C.tid; i < rank * ldx; i += C.nt) J[i] = X[i];
    __syncthreads();
    nlive = jacobi_lds(C, J, len, rank, ldx, thr2, &sw, J + rank * ldx);
    for (int i = C.tid; i < nlive * ldx; i += C.nt) X[i] = J[i];
    __syncthreads();
  } else {
    // idle pair slots use two scratch columns of pad rows in the (free) LO
    // buffer, which holds P2^2 / 2 >= 2 pad elements
    nlive = jacobi_lds(C, X, len, rank, ldx, thr2, &sw, C.LO);
  }
  ph_add(C, kPhJacobi, t0);
  if (C.tid == 0) {
    if (sw > C.sstat[1]) C.sstat[1] = sw;
    C.sstat[2] += sw;
    C.sstat[3] += 1;
    C.sstat[5] += 32LL * dl * dr * dm;  // theta = Lt . Rt (complex MACs x 8)
  }
  choose_k(C, nlive, len, capk);
  const int k = C.sk[0];
  const double inv = C.sinv[0];
  if (C.tid == 0) C.sstat[5] += 8LL * k * nc * len;  // Q^dag theta
  // Q_i = X_{perm i} / sig_{perm i}  -> LO  (len x k, column i at LO + i*len)
  sc2* Q = C.LO;
  for (DivWalk w(C.tid, C.nt, len); w.idx < k * len; w.next()) {
    const int i = w.q;
    const int r = w.r;
    const int idx = w.idx;
    const int c = C.perm[i];
    Q[idx] = cscale(X[c * ldx + r], 1.0 / C.sig[c]);
  }
  __syncthreads();
  // the unrotated theta back from HBM into the (now free) Jacobi buffer
  for (int idx = C.tid; idx < nc * ldx; idx += C.nt) X[idx] = X0[idx];
  __syncthreads();
  // Dm[i][c] = sum_r conj(Q_i[r]) theta_c[r]  -> new centre in LC
  {
    sc2* LC = C.LC;
    cgemm_mfma<kMfmaSteps>(C.tid, C.nt, k, nc, len,
               [&](int i, int r) { return cconj(Q[i * len + r]); },
               [&](int r, int c) { return X[c * ldx + r]; },
               [&](int i, int c, c2 acc) {
                 if (ltr)
                   LC[i * nc + c] = cscale(acc, inv);
                 else
                   LC[c * k + i] = cscale(cconj(acc), inv);
               });
  }
  // isometry to HBM with the finishing gate
  if (!iso) {
  } else if (ltr) {
    // site b: (dl, 2, k), A[a,s,i] = sum_t G[s][t] Q_i[a*2+t]
    const int n = dl * 2 * k;
    for (DivWalk w(C.tid, C.nt, 2 * k); w.idx < n; w.next()) {
      const int a = w.q;
      const int s = w.r >= k ? 1 : 0;
      const int i = w.r - s * k;
      const c2 q0 = Q[i * len + a * 2 + 0];
      const c2 q1 = Q[i * len + a * 2 + 1];
      iso[(size_t)(a * 2 + s) * iso_capr + i] = m22_row(Gfin, s, q0, q1);
    }
  } else {
    // site b+1: (k, 2, dr), A[i,s,c] = sum_t G[s][t] conj(Q_i[t*dr + c])
    const int n = k * 2 * dr;
    for (DivWalk w(C.tid, C.nt, 2 * dr); w.idx < n; w.next()) {
      const int i = w.q;
      const int s = w.r >= dr ? 1 : 0;
      const int c = w.r - s * dr;
      const c2 q0 = cconj(Q[i * len + c]);
      const c2 q1 = cconj(Q[i * len + dr + c]);
      iso[(size_t)(i * 2 + s) * iso_capr + c] = m22_row(Gfin, s, q0, q1);
    }
  }
  __syncthreads();
  ph_add(C, kPhFinish, t0);
  return k;
}

// ----------------------------------------------------------------------------
// Gate table entry of slice l, site j: R, dR/dux, dR/duy (12 complex).
__device__ __forceinline__ const c2* gate_ptr(const c2* gates, int N, int l, int j) {
  return gates + ((size_t)l * N + j) * 12;
}

// ----------------------------------------------------------------------------
// Gradient accumulator of one trajectory: 2 Re(conj(O) dO) into g, and dO
// itself when requested.
struct GradOut {
  double* g;  // [nctrl] 2 Re(conj O dO)
  c2* dO;     // [nctrl] or nullptr
  c2 O;
};

// Extra work of the adjoint's sweeps with Heisenberg crosstalk, where the
// u^zz derivative sits inside the ordered bond product (App. A): for the
// forward sweep of slice l, d/du^zz_b places -i dt Z_b Z_{b+1} right after
// G_b, and its matrix element pairs the forward working state just after
// bond b (alpha_b) with the backward working state just before bond b
// (beta_b), the backward slice undoing the bonds in the opposite order.
//   kSweepCentres: the forward slice re-run from its input a_l, which also
//     keeps the centre left after every bond update in `cen` (MPS layout;
//     after bond b: site b+1 sweeping left to right, site b right to left);
//     with a null dst it writes nothing else.  With the left-isometric sites (taken from
//     a_{l+1}, its post factor undone) and the untouched sites of the input
//     (pre a_l) it spells out alpha_b.
//   kSweepInsert: the backward slice (beta_b is its working state) adds
//     -i dt <beta_b| Z_b Z_{b+1} |alpha_b> before each bond b with u^zz.  The
//     environment on the side the sweep has not reached is the stored one
//     of <b_{l+1}|a_{l+1}> (site-local factors cancel in it); the one on the
//     side it has passed is grown bond by bond from the final backward sites
//     and the input sites of a_l (the pre factor cancels there).
// kSweepPlain and kSweepMid are the template argument of slice_sweep; a
// kSweepMid sweep does the work of ex->mode (kSweepCentres or kSweepInsert),
// so that both passes share one instance of the sweep.
constexpr int kSweepPlain = 0, kSweepMid = 3, kSweepCentres = 1, kSweepInsert = 2;
struct SweepExtra {
  int mode;          // kSweepCentres or kSweepInsert
  c2* cen;           // centres of the forward re-run
  const c2* a_next;  // a_{l+1} and its dims
  const int* dn;
  const c2* a_prev;  // a_l and its dims
  const int* dp;
  const c2* envs;    // <b_{l+1}|a_{l+1}>, stride cap^2: left E_j [bra][ket] for a
                     // right-to-left backward sweep, right F_j [ket][bra] otherwise
  c2* inc;           // 2 cap^2: the environment grown by the sweep (ping-pong)
  GradOut* go;
  size_t gidx;       // gradient index of u^zz (slice l, bond 0)
};

// <bra| Z_b Z_{b+1} |ket> from sites b, b+1 of each state and the
// environments on either side:
//   sum E(z,a) conj(B1[z,s,x]) (G1 A1)[a,s,y] z_s conj(B2[x,t,x']) (G2 A2)[y,t,y'] z_t Rr(x',y')
// B1 (bl,2,bm), A1 (al,2,am), B2 (bm,2,br), A2 (am,2,ar); T(i,s,j) at
// T[(i*2+s)*ld + j]; E(z,a) = Ep[z*es0 + a*es1], Rr(x',y') = Rp[x'*rs0 + y'*rs1].
// Scratch: C.X.  Returns the value to every thread.
template <class PE, class PB1, class PA1, class PB2, class PA2, class PR>
__device__ __forceinline__ c2 zz_sandwich(Ctx& C, PE Ep, int es0, int es1, PB1 B1, int ldb1, PA1 A1,
                                          int lda1, const M22& G1, PB2 B2, int ldb2, PA2 A2, int lda2,
                                          const M22& G2, PR Rp, int rs0, int rs1, int bl, int al,
                                          int bm, int am, int br, int ar) {
  int P2 = 4;
  while (P2 < 2 * C.cap) P2 <<= 1;
  const int xs = P2 * (P2 + 1);
  sc2* P = C.X;                     // P[s][z][y]   2 bl am
  sc2* Q = C.X + xs - bm * am;      // Q[x][y]      bm am (top of X)
  sc2* Wt = C.X;                    // W[t][x][y']  2 bm ar (P is dead by then)
  if (C.tid == 0) C.sstat[5] += 16LL * (bl * am * al + bm * am * bl + bm * ar * am + bm * br * ar);
  // P[s][z][y] = sum_a E(z,a) (G1 A1)[a,s,y]
  for (DivWalk w(C.tid, C.nt, am); w.idx < bl * am; w.next()) {
    const int z = w.q, y = w.r;
    c2 u0 = cmk(0.0, 0.0), u1 = cmk(0.0, 0.0);
    for (int a = 0; a < al; ++a) {
      const c2 e = Ep[z * es0 + a * es1];
      u0 = cfma(e, A1[(size_t)(a * 2 + 0) * lda1 + y], u0);
      u1 = cfma(e, A1[(size_t)(a * 2 + 1) * lda1 + y], u1);
    }
    P[z * am + y] = m22_row(G1, 0, u0, u1);
    P[bl * am + z * am + y] = m22_row(G1, 1, u0, u1);
  }
  __syncthreads();
  // Q[x][y] = sum_s z_s sum_z conj(B1[z,s,x]) P[s][z][y]
  for (DivWalk w(C.tid, C.nt, am); w.idx < bm * am; w.next()) {
    const int x = w.q, y = w.r;
    c2 q0 = cmk(0.0, 0.0), q1 = cmk(0.0, 0.0);
    for (int z = 0; z < bl; ++z) {
      q0 = cfmac(B1[(size_t)(z * 2 + 0) * ldb1 + x], P[z * am + y], q0);
      q1 = cfmac(B1[(size_t)(z * 2 + 1) * ldb1 + x], P[bl * am + z * am + y], q1);
    }
    Q[x * am + y] = csub(q0, q1);
  }
  __syncthreads();
  // W[t][x][y'] = sum_y Q[x][y] (G2 A2)[y,t,y']
  for (DivWalk w(C.tid, C.nt, ar); w.idx < bm * ar; w.next()) {
    const int x = w.q, yp = w.r;
    c2 u0 = cmk(0.0, 0.0), u1 = cmk(0.0, 0.0);
    for (int y = 0; y < am; ++y) {
      const c2 q = Q[x * am + y];
      u0 = cfma(q, A2[(size_t)(y * 2 + 0) * lda2 + yp], u0);
      u1 = cfma(q, A2[(size_t)(y * 2 + 1) * lda2 + yp], u1);
    }
    Wt[x * ar + yp] = m22_row(G2, 0, u0, u1);
    Wt[bm * ar + x * ar + yp] = m22_row(G2, 1, u0, u1);
  }
  __syncthreads();
  // sum_{t,x,x'} z_t conj(B2[x,t,x']) sum_y' W[t][x][y'] Rr(x',y')
  c2 acc[1] = {cmk(0.0, 0.0)};
  for (DivWalk w(C.tid, C.nt, br); w.idx < 2 * bm * br; w.next()) {
    const int t = w.q >= bm ? 1 : 0;
    const int x = w.q - t * bm, xp = w.r;
    c2 v = cmk(0.0, 0.0);
    for (int yp = 0; yp < ar; ++yp) v = cfma(Wt[t * bm * ar + x * ar + yp], Rp[xp * rs0 + yp * rs1], v);
    const c2 bv = B2[(size_t)(x * 2 + t) * ldb2 + xp];
    const c2 term = cmul(cconj(bv), v);
    acc[0] = t ? csub(acc[0], term) : cadd(acc[0], term);
  }
  block_sum<1>(C, acc);
  return acc[0];
}

// Right environment grown by one site: Rn[x][y] = sum_s sum_x' conj(St[x,s,x'])
// sum_y' Ap[y,s,y'] Ro[x'][y'], St (nx,2,nxo), Ap (ny,2,nyo), Ro (nxo x nyo)
// and Rn (nx x ny) packed row-major.  Scratch: C.X.
__device__ __forceinline__ void grow_right(Ctx& C, const c2* St, int lds_, const c2* Ap, int lda,
                                           const c2* Ro, c2* Rn, int nx, int nxo, int ny, int nyo) {
  sc2* T = C.X;  // T[s][y][x']
  if (C.tid == 0) C.sstat[5] += 16LL * (ny * nxo * nyo + nx * ny * nxo);
  for (DivWalk w(C.tid, C.nt, nxo); w.idx < 2 * ny * nxo; w.next()) {
    const int s = w.q >= ny ? 1 : 0;
    const int y = w.q - s * ny, xp = w.r;
    c2 v = cmk(0.0, 0.0);
    for (int yp = 0; yp < nyo; ++yp) v = cfma(Ap[(size_t)(y * 2 + s) * lda + yp], Ro[xp * nyo + yp], v);
    T[(s * ny + y) * nxo + xp] = v;
  }
  __syncthreads();
  for (DivWalk w(C.tid, C.nt, ny); w.idx < nx * ny; w.next()) {
    const int x = w.q, y = w.r;
    c2 v = cmk(0.0, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int xp = 0; xp < nxo; ++xp)
        v = cfmac(St[(size_t)(x * 2 + s) * lds_ + xp], T[(s * ny + y) * nxo + xp], v);
    Rn[x * ny + y] = v;
  }
  __syncthreads();
}

// Left environment grown by one site: Ln[x][y] = sum_s sum_x0 conj(St[x0,s,x])
// sum_y0 Lo[x0][y0] Ap[y0,s,y], St (nxo,2,nx), Ap (nyo,2,ny), Lo (nxo x nyo),
// Ln (nx x ny) packed row-major.  Scratch: C.X.
__device__ __forceinline__ void grow_left(Ctx& C, const c2* St, int lds_, const c2* Ap, int lda,
                                          const c2* Lo, c2* Ln, int nx, int nxo, int ny, int nyo) {
  sc2* T = C.X;  // T[s][x0][y]
  if (C.tid == 0) C.sstat[5] += 16LL * (nxo * ny * nyo + nx * ny * nxo);
  for (DivWalk w(C.tid, C.nt, ny); w.idx < 2 * nxo * ny; w.next()) {
    const int s = w.q >= nxo ? 1 : 0;
    const int x0 = w.q - s * nxo, y = w.r;
    c2 v = cmk(0.0, 0.0);
    for (int y0 = 0; y0 < nyo; ++y0) v = cfma(Lo[x0 * nyo + y0], Ap[(size_t)(y0 * 2 + s) * lda + y], v);
    T[(s * nxo + x0) * ny + y] = v;
  }
  __syncthreads();
  for (DivWalk w(C.tid, C.nt, ny); w.idx < nx * ny; w.next()) {
    const int x = w.q, y = w.r;
    c2 v = cmk(0.0, 0.0);
    for (int s = 0; s < 2; ++s)
      for (int x0 = 0; x0 < nxo; ++x0)
        v = cfmac(St[(size_t)(x0 * 2 + s) * lds_ + x], T[(s * nxo + x0) * ny + y], v);
    Ln[x * ny + y] = v;
  }
  __syncthreads();
}

// Centre left in LC (dl, 2, dr packed) to an MPS-layout site (row stride capr).
__device__ __forceinline__ void save_centre(Ctx& C, c2* site, int dl, int dr, int capr) {
  for (DivWalk w(C.tid, C.nt, dr); w.idx < 2 * dl * dr; w.next())
    site[(size_t)w.q * capr + w.r] = C.LC[w.idx];
}

// One slice of the two-site layer with the two half rotations fused: every
// site is rotated by G when it is first loaded and again when it is final
// for this slice, so src -> dst realises G . trunc[Z . (G psi)] (Sec. II,
// Eq. 4, second order).  Z applies the bond gates in sweep order.  For an
// adjoint slice G = R^dag and every bond gate is replaced by its adjoint
// (time t -> -t).  src may equal dst.  kX and ex: the extra work described
// at SweepExtra (dst and dst_dims may be null for the kSweepCentres pass).
template <int kX>
__device__ __forceinline__ void slice_sweep(Ctx& C, const c2* src, const int* src_dims, c2* dst,
                            int* dst_dims, bool ltr, const c2* gates, int l, bool dag,
                            double sign, const double* uzz, const double* Jrow,
                            const SweepExtra* ex) {
  const int N = C.md.N;
  const sLayout& L = *C.L;
  const int cc = C.cap * C.cap;
  for (int b = C.tid; b <= N; b += C.nt) C.sdims[b] = src_dims[b];
  __syncthreads();
  // U_l = post Z pre with post the table entry (R, or X Y in the first-order
  // split) and pre = post (second order) or I (first order); the adjoint
  // slice applies post^dag when a site is loaded and pre^dag when it is final
  const bool first = C.md.order == 1;
  M22 eye;
  eye.m[0] = cmk(1.0, 0.0); eye.m[1] = cmk(0.0, 0.0); eye.m[2] = cmk(0.0, 0.0); eye.m[3] = cmk(1.0, 0.0);
  auto gload = [&](int j) {
    const M22 g = m22_load(gate_ptr(gates, N, l, j));
    return dag ? m22_dag(g) : (first ? eye : g);
  };
  auto gfin = [&](int j) {
    const M22 g = m22_load(gate_ptr(gates, N, l, j));
    return dag ? (first ? eye : m22_dag(g)) : g;
  };
  auto bgate = [&](int b) {
    double cz = 0.0, jx = 0.0, jy = 0.0;
    if (bit(C.md.zzm, b)) cz += uzz[(size_t)l * (N - 1) + b];
    if (bit(C.md.xtm, b)) {
      if (C.md.heis) {
        jx = Jrow[3 * b];
        jy = Jrow[3 * b + 1];
        cz += Jrow[3 * b + 2];
      } else {
        cz += Jrow[b];
      }
    }
    return bond_gate(sign * C.md.dt, jx, jy, cz);
  };
  auto add_zz = [&](int b, c2 val) {
    if (C.tid == 0) {
      const c2 v = cmk(C.md.dt * val.y, -C.md.dt * val.x);  // -i dt val
      const size_t idx = ex->gidx + b;
      ex->go->g[idx] += 2.0 * (ex->go->O.x * v.x + ex->go->O.y * v.y);
      if (ex->go->dO) ex->go->dO[idx] = cadd(ex->go->dO[idx], v);
    }
  };
  const bool cen_mode = kX == kSweepMid && ex->mode == kSweepCentres;
  const bool ins_mode = kX == kSweepMid && ex->mode == kSweepInsert;
  int cur = 0;  // ping-pong half of ex->inc holding the grown environment
  if (ltr) {
    load_site(C, C.LC, src + L.off[0], 1, C.sdims[1], L.cap[1], gload(0));
    if (ins_mode && C.tid == 0) ex->inc[0] = cmk(1.0, 0.0);
    __syncthreads();
    for (int b = 0; b < N - 1; ++b) {
      const int dl = C.sdims[b], dm = C.sdims[b + 1], dr = C.sdims[b + 2];
      long long tl = ph_now(C);
      load_site(C, C.LO, src + L.off[b + 1], dm, dr, L.cap[b + 2], gload(b + 1));
      __syncthreads();
      ph_add(C, kPhLoad, tl);
      if (ins_mode && bit(C.md.zzm, b)) {
        const int* dp = ex->dp;
        const int* dn = ex->dn;
        const c2 v = zz_sandwich(C, ex->inc + cur * cc, dp[b], 1, C.LC, dm, ex->cen + L.off[b],
                                 L.cap[b + 1], eye, C.LO, dr, ex->a_next + L.off[b + 1], L.cap[b + 2],
                                 gload(b + 1), ex->envs + (size_t)(b + 2) * cc, 1, dr, dl, dp[b], dm,
                                 dn[b + 1], dr, dn[b + 2]);
        add_zz(b, v);
      }
      const int k = bond_split(C, C.LC, C.LO, dl, dm, dr, bgate(b), true,
                               dst ? dst + L.off[b] : nullptr, L.cap[b + 1], gfin(b), L.cap[b + 1]);
      if (C.tid == 0) C.sdims[b + 1] = k;
      __syncthreads();
      if (cen_mode) save_centre(C, ex->cen + L.off[b + 1], k, dr, L.cap[b + 2]);
      if (ins_mode && b < C.md.zz_hi) {
        const int* dp = ex->dp;
        grow_left(C, dst + L.off[b], L.cap[b + 1], ex->a_prev + L.off[b], L.cap[b + 1],
                  ex->inc + cur * cc, ex->inc + (1 - cur) * cc, k, dl, dp[b + 1], dp[b]);
        cur ^= 1;
      }
    }
    if (dst) store_site(C, dst + L.off[N - 1], C.LC, C.sdims[N - 1], 1, L.cap[N], gfin(N - 1));
  } else {
    load_site(C, C.LC, src + L.off[N - 1], C.sdims[N - 1], 1, L.cap[N], gload(N - 1));
    if (ins_mode && C.tid == 0) ex->inc[0] = cmk(1.0, 0.0);
    __syncthreads();
    for (int b = N - 2; b >= 0; --b) {
      const int dl = C.sdims[b], dm = C.sdims[b + 1], dr = C.sdims[b + 2];
      long long tl = ph_now(C);
      load_site(C, C.LO, src + L.off[b], dl, dm, L.cap[b + 1], gload(b));
      __syncthreads();
      ph_add(C, kPhLoad, tl);
      if (ins_mode && bit(C.md.zzm, b)) {
        const int* dp = ex->dp;
        const int* dn = ex->dn;
        const c2 v = zz_sandwich(C, ex->envs + (size_t)b * cc, dn[b], 1, C.LO, dm,
                                 ex->a_next + L.off[b], L.cap[b + 1], gload(b), C.LC, dr,
                                 ex->cen + L.off[b + 1], L.cap[b + 2], eye, ex->inc + cur * cc,
                                 dp[b + 2], 1, dl, dn[b], dm, dn[b + 1], dr, dp[b + 2]);
        add_zz(b, v);
      }
      const int k = bond_split(C, C.LO, C.LC, dl, dm, dr, bgate(b), false,
                               dst ? dst + L.off[b + 1] : nullptr, L.cap[b + 2], gfin(b + 1),
                               L.cap[b + 1]);
      if (C.tid == 0) C.sdims[b + 1] = k;
      __syncthreads();
      if (cen_mode) save_centre(C, ex->cen + L.off[b], dl, k, L.cap[b + 1]);
      if (ins_mode && b > C.md.zz_lo) {
        const int* dp = ex->dp;
        grow_right(C, dst + L.off[b + 1], L.cap[b + 2], ex->a_prev + L.off[b + 1], L.cap[b + 2],
                   ex->inc + cur * cc, ex->inc + (1 - cur) * cc, k, dr, dp[b + 1], dp[b + 2]);
        cur ^= 1;
      }
    }
    if (dst) store_site(C, dst + L.off[0], C.LC, 1, C.sdims[1], L.cap[1], gfin(0));
  }
  __syncthreads();
  if (dst_dims)
    for (int b = C.tid; b <= N; b += C.nt) dst_dims[b] = C.sdims[b];
  __syncthreads();
}

// Forward slice l (0-based): left to right when M - 1 - l is odd, so the
// last slice sweeps right to left and every forward slice runs opposite to
// its adjoint (the bond visited first acts first).
__device__ __forceinline__ bool forward_ltr(const Ctx& C, int l) { return ((C.md.M - 1 - l) % 2) == 1; }
__device__ __forceinline__ void forward_slice(Ctx& C, const c2* src, const int* sd, c2* dst,
                                              int* dd, const c2* gates, int l,
                                              const double* uzz, const double* Jrow) {
  slice_sweep<kSweepPlain>(C, src, sd, dst, dd, forward_ltr(C, l), gates, l, false, 1.0, uzz, Jrow,
                           nullptr);
}
// Adjoint slice l (0-based): b_l = U_l^dag b_{l+1}; left to right when
// M - 1 - l is even.
__device__ __forceinline__ void adjoint_slice(Ctx& C, const c2* src, const int* sd, c2* dst,
                                              int* dd, const c2* gates, int l,
                                              const double* uzz, const double* Jrow) {
  slice_sweep<kSweepPlain>(C, src, sd, dst, dd, !forward_ltr(C, l), gates, l, true, -1.0, uzz,
                           Jrow, nullptr);
}
// Adjoint slice l with the mid-sweep u^zz insertions: forward slice l re-run
// from a_l (ex.a_prev) keeping its centres, then the backward slice of b (in
// place) with the insertions; one instance of the sweep serves both passes.
__device__ __forceinline__ void adjoint_slice_mid(Ctx& C, c2* b, int* bd, const c2* gates, int l,
                                                  const double* uzz, const double* Jrow,
                                                  SweepExtra& ex) {
  const bool fl = forward_ltr(C, l);
  for (int pass = 0; pass < 2; ++pass) {
    const bool ins = pass == 1;
    ex.mode = ins ? kSweepInsert : kSweepCentres;
    slice_sweep<kSweepMid>(C, ins ? b : ex.a_prev, ins ? bd : ex.dp, ins ? b : nullptr,
                           ins ? bd : nullptr, ins ? !fl : fl, gates, l, ins, ins ? -1.0 : 1.0,
                           uzz, Jrow, &ex);
  }
}

// Copy one MPS between two capacity layouts (dims must fit the destination).
__device__ __forceinline__ void copy_mps(Ctx& C, const c2* src, const int* sdims_g, int sdcap, c2* dst,
                         int* ddims_g, const sLayout& Ld) {
  const int N = C.md.N;
  for (int b = C.tid; b <= N; b += C.nt) {
    int d = sdims_g[b];
    const int lim = min(Ld.cap[b], bond_cap(N, sdcap, b));
    if (d > lim || d < 1 || ((b == 0 || b == N) && d != 1)) {
      flag_or(C, 1);
      d = max(1, min(d, lim));
      if (b == 0 || b == N) d = 1;
    }
    C.sdims[b] = d;
    ddims_g[b] = d;
  }
  __syncthreads();
  long long soff = 0;
  for (int j = 0; j < N; ++j) {
    const int dl = C.sdims[j], dr = C.sdims[j + 1];
    const int scr = bond_cap(N, sdcap, j + 1);
    const int n = dl * 2 * dr;
    for (DivWalk w(C.tid, C.nt, dr); w.idx < n; w.next()) {
      const int row = w.q, c = w.r;
      dst[Ld.off[j] + (size_t)row * Ld.cap[j + 1] + c] = src[soff + (size_t)row * scr + c];
    }
    soff += (long long)bond_cap(N, sdcap, j) * 2 * scr;
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// Transfer environments between bra and ket (each with its own layout).
// LDS scratch (complex, cap = max capacity): E, F, Ep (cap^2 each), TF, TFp
// (2 cap^2 each) -> 7 cap^2, aliased on LC/LO/X.
struct EnvBufs {
  sc2 *E, *F, *Ep, *TF, *TFp;
};
__device__ __forceinline__ EnvBufs env_bufs(Ctx& C) {
  const int c2n = C.cap * C.cap;
  EnvBufs e;
  e.E = C.LC;
  e.F = C.LC + c2n;
  e.Ep = C.LO;
  e.TF = C.X;
  e.TFp = C.X + 2 * c2n;
  return e;
}

// Left pass: E_{j+1} = sum_s B_j[s]^dag E_j A_j[s]; stores E_j (j = 0..N) to
// envs (stride cap^2) when envs != nullptr.  Returns E_N = <bra|ket>.
__device__ __forceinline__ c2 left_envs(Ctx& C, const c2* bra, const int* bd, const sLayout& Lb,
                        const c2* ket, const int* kd, const sLayout& Lk, c2* envs) {
  const int N = C.md.N;
  const int cc = C.cap * C.cap;
  EnvBufs eb = env_bufs(C);
  if (C.tid == 0) eb.E[0] = cmk(1.0, 0.0);
  __syncthreads();
  for (int j = 0; j < N; ++j) {
    const int bl = bd[j], br = bd[j + 1], al = kd[j], ar = kd[j + 1];
    if (envs)
      for (int idx = C.tid; idx < bl * al; idx += C.nt) envs[(size_t)j * cc + idx] = eb.E[idx];
    const c2* A = ket + Lk.off[j];
    const int acap = Lk.cap[j + 1];
    const c2* Bt = bra + Lb.off[j];
    const int bcap = Lb.cap[j + 1];
    if (C.tid == 0) C.sstat[5] += 16LL * (bl * ar * al + br * ar * bl);
    // T[s][z][y] = sum_w E[z][w] A[w,s,y]: bl x (2 ar), column (s, y)
    {
      sc2* E = eb.E;
      sc2* TF = eb.TF;
      cgemm_mfma<kMfmaSteps>(C.tid, C.nt, bl, 2 * ar, al,
                 [&](int z, int w) { return E[z * al + w]; },
                 [&](int w, int c) {
                   const int s = c >= ar ? 1 : 0;
                   return A[(size_t)(w * 2 + s) * acap + c - s * ar];
                 },
                 [&](int z, int c, c2 v) {
                   const int s = c >= ar ? 1 : 0;
                   TF[s * cc + z * ar + c - s * ar] = v;
                 });
    }
    __syncthreads();
    // E'[x][y] = sum_{s,z} conj(B[z,s,x]) T[s][z][y]: br x ar, depth (s, z)
    {
      sc2* E = eb.E;
      sc2* TF = eb.TF;
      cgemm_mfma<kMfmaSteps>(C.tid, C.nt, br, ar, 2 * bl,
                 [&](int x, int q) {
                   const int s = q >= bl ? 1 : 0;
                   return cconj(Bt[(size_t)((q - s * bl) * 2 + s) * bcap + x]);
                 },
                 [&](int q, int y) {
                   const int s = q >= bl ? 1 : 0;
                   return TF[s * cc + (q - s * bl) * ar + y];
                 },
                 [&](int x, int y, c2 v) { E[x * ar + y] = v; });
    }
    __syncthreads();
  }
  if (envs && C.tid == 0) envs[(size_t)N * cc] = eb.E[0];
  const c2 out = eb.E[0];
  __syncthreads();
  return out;
}

}  // namespace TNRG_NS
