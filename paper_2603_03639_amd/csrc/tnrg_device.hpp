// Device building blocks of the MPS robust-GRAPE hot path for gfx950.
//
// One workgroup owns one trajectory (one crosstalk sample k and one input r).
// Everything a bond update touches lives in LDS: the two site tensors, the
// two-site matrix theta and the one-sided Jacobi working copy.  The MPS itself
// lives in HBM in a fixed-capacity layout (see include/tnrg.h) and is streamed
// site by site during a sweep, so a slice reads and writes every site once.
//
// Method references (Le, Mintert, Ginossar): second-order slice of Sec. II,
// Eq. 4 with SVD compression to a maximum bond size; ensemble state fidelity
// of Sec. II, Eq. 7; adjoint gradient of App. A, Eqs. A1-A2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnrg {

typedef double2 c2;

constexpr int kMaxSites = 256;
constexpr int kMaxWaves = 16;

// ----------------------------------------------------------------------------
// complex helpers (double2: x = real, y = imaginary)
__device__ __forceinline__ c2 cmk(double r, double i) { return make_double2(r, i); }
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
  uint64_t zzm[4];  // bit b: bond b carries u^zz
  uint64_t xtm[4];  // bit b: bond b carries crosstalk J
};
__device__ __forceinline__ bool bit(const uint64_t* m, int b) {
  return (m[b >> 6] >> (b & 63)) & 1ull;
}

// Capacity of bond b: min(dcap, 2^b, 2^(N-b)).
__host__ __device__ __forceinline__ int bond_cap(int N, int dcap, int b) {
  int c = dcap;
  if (b < 30 && (1 << b) < c) c = 1 << b;
  int rb = N - b;
  if (rb < 30 && (1 << rb) < c) c = 1 << rb;
  return c;
}

// Fixed-capacity MPS layout, built in LDS at kernel start.
struct Layout {
  int N;
  int dcap;
  int cap[kMaxSites + 1];
  long long off[kMaxSites + 1];  // off[N] = elements per trajectory
};
__device__ void layout_build(Layout& L, int N, int dcap) {
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
__host__ __device__ inline long long site_offset_slow(int N, int dcap, int j) {
  long long o = 0;
  for (int i = 0; i < j; ++i) o += (long long)bond_cap(N, dcap, i) * 2 * bond_cap(N, dcap, i + 1);
  return o;
}

// Per-workgroup context.  LDS buffers are sized from the capacity `cap`:
//   LC, LO : 2 cap^2 complex  (centre tensor, other tensor / isometry Q)
//   X      : 2 cap (2 cap + 1) complex (Jacobi working matrix)
//   sig    : 2 cap doubles, perm : 2 cap ints
struct Ctx {
  int tid, nt;
  int cap;
  c2* LC;
  c2* LO;
  c2* X;
  double* sig;
  int* perm;
  c2* X0;       // global scratch (2 cap (2 cap + 1)), the unrotated theta
  Layout* L;    // layout of the internal states
  int* sdims;   // LDS [kMaxSites + 1]
  ModelDev md;
  // per-trajectory bookkeeping in LDS (written by thread 0)
  int* sflag;
  // [8]: max dim, max sweeps, total sweeps, svd count, Jacobi flops,
  // contraction flops (theta, projection, environments), unused x2
  long long* sstat;
  double* red;       // LDS [kMaxWaves * 8]
  int* sk;           // LDS scalar: kept singular values of the last split
  double* sinv;      // LDS scalar: 1 / norm of kept singular values
};

// ----------------------------------------------------------------------------
// Block-wide deterministic reduction of V complex values (V <= 4).  Every
// thread passes its partial sums; the result is returned to every thread.
// The summation order is fixed (butterfly inside each wave, waves in order).
template <int V>
__device__ void block_sum(Ctx& C, c2 (&v)[V]) {
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
// One-sided (Hestenes) Jacobi SVD of the len x nc matrix X held column-major
// in LDS (column c at X + c*ldx).  Columns are rotated pairwise until every
// pair is orthogonal to tol = len * 2^-52 relative to the column norms; the
// columns then hold sigma_i u_i.  Pairs are visited in the round-robin
// (circle) order, all disjoint pairs of a round in parallel; each pair's rows
// are split over LPP lanes whose partial dot products are combined by a
// butterfly, so every lane of the pair derives the same rotation.
// Writes sig[c] = ||X_c||; returns the number of sweeps.
__device__ int jacobi_lds(Ctx& C, c2* X, int len, int nc, int ldx) {
  const int tid = C.tid, NT = C.nt;
  const int P = (nc + 1) >> 1;
  const int np = 2 * P, m = np - 1;
  int LPP = 1;
  while (LPP < 16 && P * LPP * 2 <= NT) LPP <<= 1;
  const int slots = NT / LPP;
  const int p_local = tid / LPP, q = tid % LPP;
  const double tol = (double)len * 2.220446049250313e-16;
  int sweeps = 0;
  const int max_sweeps = C.md.max_sweeps;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    int rotated = 0;
    for (int r = 0; r < m; ++r) {
      for (int pbase = 0; pbase < P; pbase += slots) {
        const int pp = pbase + p_local;
        int ci = 0, cj = 0;
        bool valid = (p_local < slots) && (pp < P);
        if (valid) {
          if (pp == 0) {
            ci = 0;
            cj = 1 + (r % m);
          } else {
            ci = 1 + (r + pp) % m;
            cj = 1 + (r - pp + m) % m;
          }
          valid = (ci < nc) && (cj < nc);
        }
        double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
        if (valid) {
          const c2* xc = X + ci * ldx;
          const c2* yc = X + cj * ldx;
          for (int row = q; row < len; row += LPP) {
            c2 x = xc[row], y = yc[row];
            a = fma(x.x, x.x, fma(x.y, x.y, a));
            b = fma(y.x, y.x, fma(y.y, y.y, b));
            gr = fma(x.x, y.x, fma(x.y, y.y, gr));
            gi = fma(x.x, y.y, fma(-x.y, y.x, gi));
          }
        }
        for (int o = 1; o < LPP; o <<= 1) {
          a += __shfl_xor(a, o, 64);
          b += __shfl_xor(b, o, 64);
          gr += __shfl_xor(gr, o, 64);
          gi += __shfl_xor(gi, o, 64);
        }
        if (valid && a > 0.0 && b > 0.0) {
          const double ag = sqrt(fma(gr, gr, gi * gi));
          if (ag > tol * sqrt(a * b)) {
            rotated = 1;
            const double zeta = (b - a) / (2.0 * ag);
            double t;
            if (fabs(zeta) > 1e100)
              t = 0.5 / zeta;
            else
              t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
            const double cs = 1.0 / sqrt(fma(t, t, 1.0));
            const double sn = cs * t;
            const double er = gr / ag, ei = gi / ag;  // e = gamma / |gamma|
            // x' = c x - s conj(e) y,  y' = s e x + c y
            const double pr = sn * er, pi = sn * ei;  // s e
            c2* xc = X + ci * ldx;
            c2* yc = X + cj * ldx;
            for (int row = q; row < len; row += LPP) {
              c2 x = xc[row], y = yc[row];
              c2 xn, yn;
              // conj(s e) y = (pr - i pi)(y.x + i y.y)
              xn.x = cs * x.x - (pr * y.x + pi * y.y);
              xn.y = cs * x.y - (pr * y.y - pi * y.x);
              // (s e) x = (pr + i pi)(x.x + i x.y)
              yn.x = cs * y.x + (pr * x.x - pi * x.y);
              yn.y = cs * y.y + (pr * x.y + pi * x.x);
              xc[row] = xn;
              yc[row] = yn;
            }
          }
        } else if (valid && !(a == a && b == b)) {
          // non-finite column: record and stop rotating this pair
          atomicOr(C.sflag, 4);
        }
      }
      __syncthreads();
    }
    ++sweeps;
    if (tid == 0) C.sstat[4] += 18LL * len * nc * (nc - 1);
    if (!__syncthreads_or(rotated)) break;
    if (sw + 1 == max_sweeps && tid == 0) atomicOr(C.sflag, 2);
  }
  for (int c = tid; c < nc; c += NT) {
    const c2* xc = X + c * ldx;
    double s = 0.0;
    for (int row = 0; row < len; ++row) s += cabs2(xc[row]);
    C.sig[c] = sqrt(s);
  }
  __syncthreads();
  return sweeps;
}

// Sort singular values (descending, ties by column index), choose the kept
// count k by the truncation rule and compute 1/||sigma_{1..k}||.
__device__ void choose_k(Ctx& C, int nc, int len, int capk) {
  for (int c = C.tid; c < nc; c += C.nt) {
    double v = C.sig[c];
    if (!(v == v)) v = -1.0;
    int rank = 0;
    for (int d = 0; d < nc; ++d) {
      double w = C.sig[d];
      if (!(w == w)) w = -1.0;
      rank += (w > v) || (w == v && d < c);
    }
    C.perm[rank] = c;
  }
  __syncthreads();
  if (C.tid == 0) {
    const double smax = C.sig[C.perm[0]];
    int cnt = 0;
    for (int c = 0; c < nc; ++c) cnt += (C.sig[c] >= C.md.eps * smax) ? 1 : 0;
    int k = cnt < C.md.chi ? cnt : C.md.chi;
    if (k < 1) k = 1;
    const int lim = len < nc ? len : nc;
    if (k > lim) k = lim;
    if (k > capk) {
      atomicOr(C.sflag, 1);
      k = capk;
    }
    double s2 = 0.0;
    for (int i = 0; i < k; ++i) {
      const double s = C.sig[C.perm[i]];
      s2 += s * s;
    }
    if (!(smax > 0.0) || !(s2 == s2)) atomicOr(C.sflag, 4);
    C.sk[0] = k;
    C.sinv[0] = (C.md.renorm && s2 > 0.0) ? 1.0 / sqrt(s2) : 1.0;
    if (k > C.sstat[0]) C.sstat[0] = k;
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// Site tensor transfer between HBM (capacity layout) and LDS (packed), with a
// single-site 2x2 gate applied on the physical index: out[a,s,c] = sum_t
// G[s][t] in[a,t,c].
__device__ void load_site(Ctx& C, c2* dst, const c2* site, int dl, int dr, int capr,
                          const M22& G) {
  const int n = dl * 2 * dr;
  for (int idx = C.tid; idx < n; idx += C.nt) {
    const int a = idx / (2 * dr);
    const int rem = idx - a * 2 * dr;
    const int s = rem / dr;
    const int c = rem - s * dr;
    const c2 x0 = site[(size_t)(a * 2 + 0) * capr + c];
    const c2 x1 = site[(size_t)(a * 2 + 1) * capr + c];
    dst[idx] = cfma(G.m[2 * s + 1], x1, cmul(G.m[2 * s], x0));
  }
}
__device__ void store_site(Ctx& C, c2* site, const c2* src, int dl, int dr, int capr,
                           const M22& G) {
  const int n = dl * 2 * dr;
  for (int idx = C.tid; idx < n; idx += C.nt) {
    const int a = idx / (2 * dr);
    const int rem = idx - a * 2 * dr;
    const int s = rem / dr;
    const int c = rem - s * dr;
    const c2 x0 = src[(a * 2 + 0) * dr + c];
    const c2 x1 = src[(a * 2 + 1) * dr + c];
    site[(size_t)(a * 2 + s) * capr + c] = cfma(G.m[2 * s + 1], x1, cmul(G.m[2 * s], x0));
  }
}

// ----------------------------------------------------------------------------
// Two-site update of one bond (Sec. II: apply the two-qubit gate, split by an
// SVD, compress).  Lt (dl,2,dm) and Rt (dm,2,dr) are packed in LDS; the gate
// is the ZZ phase exp(-i phi z_s z_s').
//   ltr: left factor U (left-isometric) is written to `iso` (site b, capacity
//        row stride iso_capr) after the gate Gfin, the centre diag(s) V^dag
//        (k,2,dr) is left in LC.
//   rtl: right factor V^dag is written to `iso` (site b+1), the centre
//        U diag(s) (dl,2,k) is left in LC.
// Returns k, the new bond dimension.
__device__ int bond_split(Ctx& C, const c2* Lt, const c2* Rt, int dl, int dm, int dr,
                          double phi, bool ltr, c2* iso, int iso_capr, const M22& Gfin,
                          int capk) {
  const int len = ltr ? 2 * dl : 2 * dr;
  const int nc = ltr ? 2 * dr : 2 * dl;
  const int ldx = len | 1;
  c2* X = C.X;
  c2* X0 = C.X0;
  const double cp = cos(phi), sp = sin(phi);
  const c2 ph_same = cmk(cp, -sp);  // exp(-i phi)   (z_s z_s' = +1)
  const c2 ph_diff = cmk(cp, sp);   // exp(+i phi)   (z_s z_s' = -1)
  // theta[(a,s),(s',c)] = P[s][s'] sum_b Lt[a,s,b] Rt[b,s',c]
  const int nth = 4 * dl * dr;
  for (int idx = C.tid; idx < nth; idx += C.nt) {
    const int row = idx / (2 * dr);
    const int col = idx - row * 2 * dr;
    const int s = row & 1;
    const int s2 = col / dr;
    const int c = col - s2 * dr;
    const c2* lp = Lt + row * dm;
    const c2* rp = Rt + s2 * dr + c;
    c2 acc = cmk(0.0, 0.0);
    for (int b = 0; b < dm; ++b) acc = cfma(lp[b], rp[b * 2 * dr], acc);
    acc = cmul(acc, s == s2 ? ph_same : ph_diff);
    if (ltr) {
      X[col * ldx + row] = acc;
      X0[col * ldx + row] = acc;
    } else {
      X[row * ldx + col] = cconj(acc);
      X0[row * ldx + col] = cconj(acc);
    }
  }
  __syncthreads();
  const int sw = jacobi_lds(C, X, len, nc, ldx);
  if (C.tid == 0) {
    if (sw > C.sstat[1]) C.sstat[1] = sw;
    C.sstat[2] += sw;
    C.sstat[3] += 1;
    C.sstat[5] += 32LL * dl * dr * dm;  // theta = Lt . Rt (complex MACs x 8)
  }
  choose_k(C, nc, len, capk);
  const int k = C.sk[0];
  const double inv = C.sinv[0];
  if (C.tid == 0) C.sstat[5] += 8LL * k * nc * len;  // Q^dag theta
  // Q_i = X_{perm i} / sig_{perm i}  -> LO  (len x k, column i at LO + i*len)
  c2* Q = C.LO;
  for (int idx = C.tid; idx < k * len; idx += C.nt) {
    const int i = idx / len;
    const int r = idx - i * len;
    const int c = C.perm[i];
    Q[idx] = cscale(X[c * ldx + r], 1.0 / C.sig[c]);
  }
  __syncthreads();
  // Dm[i][c] = sum_r conj(Q_i[r]) X0_c[r]  -> new centre in LC
  for (int idx = C.tid; idx < k * nc; idx += C.nt) {
    const int i = idx / nc;
    const int c = idx - i * nc;
    const c2* qi = Q + i * len;
    const c2* xc = X0 + c * ldx;
    c2 acc = cmk(0.0, 0.0);
    for (int r = 0; r < len; ++r) acc = cfmac(qi[r], xc[r], acc);
    if (ltr)
      C.LC[i * nc + c] = cscale(acc, inv);
    else
      C.LC[c * k + i] = cscale(cconj(acc), inv);
  }
  // isometry to HBM with the finishing gate
  if (ltr) {
    // site b: (dl, 2, k), A[a,s,i] = sum_t G[s][t] Q_i[a*2+t]
    const int n = dl * 2 * k;
    for (int idx = C.tid; idx < n; idx += C.nt) {
      const int a = idx / (2 * k);
      const int rem = idx - a * 2 * k;
      const int s = rem / k;
      const int i = rem - s * k;
      const c2 q0 = Q[i * len + a * 2 + 0];
      const c2 q1 = Q[i * len + a * 2 + 1];
      iso[(size_t)(a * 2 + s) * iso_capr + i] = cfma(Gfin.m[2 * s + 1], q1, cmul(Gfin.m[2 * s], q0));
    }
  } else {
    // site b+1: (k, 2, dr), A[i,s,c] = sum_t G[s][t] conj(Q_i[t*dr + c])
    const int n = k * 2 * dr;
    for (int idx = C.tid; idx < n; idx += C.nt) {
      const int i = idx / (2 * dr);
      const int rem = idx - i * 2 * dr;
      const int s = rem / dr;
      const int c = rem - s * dr;
      const c2 q0 = cconj(Q[i * len + c]);
      const c2 q1 = cconj(Q[i * len + dr + c]);
      iso[(size_t)(i * 2 + s) * iso_capr + c] = cfma(Gfin.m[2 * s + 1], q1, cmul(Gfin.m[2 * s], q0));
    }
  }
  __syncthreads();
  return k;
}

// ----------------------------------------------------------------------------
// Gate table entry of slice l, site j: R, dR/dux, dR/duy (12 complex).
__device__ __forceinline__ const c2* gate_ptr(const c2* gates, int N, int l, int j) {
  return gates + ((size_t)l * N + j) * 12;
}

// One slice of the ZZ layer with the two half rotations fused: every site is
// rotated by G when it is first loaded and again when it is final for this
// slice, so src -> dst realises G . trunc[Z . (G psi)] (Sec. II, Eq. 4, second
// order).  For an adjoint slice G = R^dag and phi -> -phi.  src may equal dst.
__device__ void slice_sweep(Ctx& C, const c2* src, const int* src_dims, c2* dst,
                            int* dst_dims, bool ltr, const c2* gates, int l, bool dag,
                            double sign, const double* uzz, const double* Jrow) {
  const int N = C.md.N;
  const Layout& L = *C.L;
  for (int b = C.tid; b <= N; b += C.nt) C.sdims[b] = src_dims[b];
  __syncthreads();
  auto gate = [&](int j) {
    M22 g = m22_load(gate_ptr(gates, N, l, j));
    return dag ? m22_dag(g) : g;
  };
  auto phase = [&](int b) {
    double c = 0.0;
    if (bit(C.md.zzm, b)) c += uzz[(size_t)l * (N - 1) + b];
    if (bit(C.md.xtm, b)) c += Jrow[b];
    return sign * C.md.dt * c;
  };
  if (ltr) {
    load_site(C, C.LC, src + L.off[0], 1, C.sdims[1], L.cap[1], gate(0));
    __syncthreads();
    for (int b = 0; b < N - 1; ++b) {
      const int dl = C.sdims[b], dm = C.sdims[b + 1], dr = C.sdims[b + 2];
      load_site(C, C.LO, src + L.off[b + 1], dm, dr, L.cap[b + 2], gate(b + 1));
      __syncthreads();
      const int k = bond_split(C, C.LC, C.LO, dl, dm, dr, phase(b), true,
                               dst + L.off[b], L.cap[b + 1], gate(b), L.cap[b + 1]);
      if (C.tid == 0) C.sdims[b + 1] = k;
      __syncthreads();
    }
    store_site(C, dst + L.off[N - 1], C.LC, C.sdims[N - 1], 1, L.cap[N], gate(N - 1));
  } else {
    load_site(C, C.LC, src + L.off[N - 1], C.sdims[N - 1], 1, L.cap[N], gate(N - 1));
    __syncthreads();
    for (int b = N - 2; b >= 0; --b) {
      const int dl = C.sdims[b], dm = C.sdims[b + 1], dr = C.sdims[b + 2];
      load_site(C, C.LO, src + L.off[b], dl, dm, L.cap[b + 1], gate(b));
      __syncthreads();
      const int k = bond_split(C, C.LO, C.LC, dl, dm, dr, phase(b), false,
                               dst + L.off[b + 1], L.cap[b + 2], gate(b + 1), L.cap[b + 1]);
      if (C.tid == 0) C.sdims[b + 1] = k;
      __syncthreads();
    }
    store_site(C, dst + L.off[0], C.LC, 1, C.sdims[1], L.cap[1], gate(0));
  }
  __syncthreads();
  for (int b = C.tid; b <= N; b += C.nt) dst_dims[b] = C.sdims[b];
  __syncthreads();
}

// Forward slice l (0-based): left to right when l is even.
__device__ __forceinline__ void forward_slice(Ctx& C, const c2* src, const int* sd, c2* dst,
                                              int* dd, const c2* gates, int l,
                                              const double* uzz, const double* Jrow) {
  slice_sweep(C, src, sd, dst, dd, (l % 2) == 0, gates, l, false, 1.0, uzz, Jrow);
}
// Adjoint slice l (0-based): b_l = U_l^dag b_{l+1}; left to right when
// M - 1 - l is even.
__device__ __forceinline__ void adjoint_slice(Ctx& C, const c2* src, const int* sd, c2* dst,
                                              int* dd, const c2* gates, int l,
                                              const double* uzz, const double* Jrow) {
  slice_sweep(C, src, sd, dst, dd, ((C.md.M - 1 - l) % 2) == 0, gates, l, true, -1.0, uzz,
              Jrow);
}

// Copy one MPS between two capacity layouts (dims must fit the destination).
__device__ void copy_mps(Ctx& C, const c2* src, const int* sdims_g, int sdcap, c2* dst,
                         int* ddims_g, const Layout& Ld) {
  const int N = C.md.N;
  for (int b = C.tid; b <= N; b += C.nt) {
    int d = sdims_g[b];
    const int lim = min(Ld.cap[b], bond_cap(N, sdcap, b));
    if (d > lim || d < 1 || ((b == 0 || b == N) && d != 1)) {
      atomicOr(C.sflag, 1);
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
    for (int idx = C.tid; idx < n; idx += C.nt) {
      const int row = idx / dr, c = idx - row * dr;
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
  c2 *E, *F, *Ep, *TF, *TFp;
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
__device__ c2 left_envs(Ctx& C, const c2* bra, const int* bd, const Layout& Lb,
                        const c2* ket, const int* kd, const Layout& Lk, c2* envs) {
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
    // T[s][z][y] = sum_w E[z][w] A[w,s,y]   (bl x ar)
    for (int idx = C.tid; idx < 2 * bl * ar; idx += C.nt) {
      const int s = idx / (bl * ar);
      const int rem = idx - s * bl * ar;
      const int z = rem / ar, y = rem - z * ar;
      c2 acc = cmk(0.0, 0.0);
      for (int w = 0; w < al; ++w) acc = cfma(eb.E[z * al + w], A[(size_t)(w * 2 + s) * acap + y], acc);
      eb.TF[s * cc + z * ar + y] = acc;
    }
    __syncthreads();
    // E'[x][y] = sum_s sum_z conj(B[z,s,x]) T[s][z][y]   (br x ar)
    for (int idx = C.tid; idx < br * ar; idx += C.nt) {
      const int x = idx / ar, y = idx - x * ar;
      c2 acc = cmk(0.0, 0.0);
      for (int s = 0; s < 2; ++s)
        for (int z = 0; z < bl; ++z)
          acc = cfmac(Bt[(size_t)(z * 2 + s) * bcap + x], eb.TF[s * cc + z * ar + y], acc);
      eb.E[idx] = acc;
    }
    __syncthreads();
  }
  if (envs && C.tid == 0) envs[(size_t)N * cc] = eb.E[0];
  const c2 out = eb.E[0];
  __syncthreads();
  return out;
}

}  // namespace tnrg
