/*
 * tnrg.h -- C ABI of the MI355X (gfx950) hot path of ensemble-robust GRAPE on
 * qubit-chain matrix product states.
 *
 * The method (Le, Mintert, Ginossar, "Mitigating many-body quantum crosstalk
 * with tensor-network robust control"):
 *   - a chain of N qubits under H(t) = sum_j [u^x_j(t) X_j + u^y_j(t) Y_j]/2
 *     + sum_b c_b(t) Z_b Z_{b+1}, with c_b = zz_mask_b u^zz_b(t)
 *     + xt_mask_b J_b  (Sec. III, Eqs. 8-9, ZZ part of the crosstalk);
 *   - piecewise-constant controls on M slices of length dt, each slice
 *     applied as the second-order split U_l = R_l Z_l R_l with
 *     R_l = exp(-i dt/2 sum_j h_j), Z_l = exp(-i dt sum_b c_b Z_b Z_{b+1}),
 *     or (split_order = 1) as the first-order product U_l = X_l Y_l Z_l of
 *     Sec. II, Eq. 4 with X_l = exp(-i dt sum_j u^x_j X_j / 2) and
 *     Y_l = exp(-i dt sum_j u^y_j Y_j / 2);
 *   - the state is an MPS (Sec. II), the ZZ layer is applied by a bond sweep
 *     with an SVD after every bond, compressed to at most chi singular values:
 *     keep k = max(1, min(chi, #{sigma_i >= trunc_eps * sigma_1})) and, with
 *     renormalize != 0, rescale the kept values to unit 2-norm;
 *   - objective: F = 1/(K R) sum_{k,r} |<T_r|psi_kr(T)>|^2 over K crosstalk
 *     samples and R input states (Sec. II, Eq. 7);
 *   - gradient: the adjoint sweep of App. A (Eqs. A1-A2), with the exact
 *     insertion operators of the chosen split.
 *
 * Conventions
 *   - Sites j = 0..N-1, bond b couples (b, b+1); |0> is the Z = +1 state.
 *   - Slice index l = 0..M-1 (0-based).  Controls are row-major float64:
 *     ux[l][j], uy[l][j] ([M][N]) and uzz[l][b] ([M][N-1]).
 *   - Trajectory t of a K x R ensemble is (k, r) = (t / R, t % R).
 *   - Complex numbers are tnrg_c128 {re, im} (the storage of complex128).
 *   - <bra|ket> is conjugate-linear in bra.
 *
 * Ownership and errors
 *   - The caller owns every buffer, including the workspace; the library
 *     allocates no device memory, keeps no pointer past a call and keeps
 *     only a per-process launch plan cache.
 *   - Every compute call is asynchronous on the given HIP stream
 *     (tnrg_stream is a hipStream_t; NULL is the default stream).
 *   - Argument errors return a negative status at once and set the
 *     thread-local message tnrg_last_error().  Device-side conditions (bond
 *     capacity exceeded, Jacobi not converged, non-finite values) are written
 *     as per-trajectory flags into the workspace; tnrg_status() synchronises
 *     the stream and reads them.
 *   - No C++ exception crosses this interface.
 */
#ifndef TNRG_H
#define TNRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} tnrg_c128;

typedef void *tnrg_stream; /* a hipStream_t */

enum {
  TNRG_OK = 0,
  TNRG_EINVAL = -1,     /* bad argument */
  TNRG_ENOMEM = -2,     /* workspace too small */
  TNRG_EHIP = -3,       /* HIP runtime error */
  TNRG_ENOCONV = -4,    /* Jacobi SVD hit max_sweeps (device flag) */
  TNRG_ENONFINITE = -5, /* non-finite value met (device flag) */
  TNRG_EOVERFLOW = -6,  /* a bond needed more than the capacity dcap */
  TNRG_EUNSUPPORTED = -7,
  TNRG_ESTALE = -8      /* grape_backward without its grape_forward (device flag) */
};

/* Device status flag bits (per trajectory, in the workspace). */
enum {
  TNRG_FLAG_OVERFLOW = 1,
  TNRG_FLAG_NOCONV = 2,
  TNRG_FLAG_NONFINITE = 4,
  TNRG_FLAG_STALE = 8
};

/* Problem statement (Sec. II-III).  Host struct; the masks are host arrays. */
typedef struct {
  int32_t n;              /* qubits N, 2 <= N <= 256 */
  int32_t m;              /* slices M >= 1 */
  double dt;              /* slice length T / M */
  int32_t chi;            /* maximum bond dimension (Sec. II, D_max) */
  double trunc_eps;       /* relative singular-value cutoff, e.g. 1e-12 */
  int32_t renormalize;    /* 1: rescale kept singular values to unit norm */
  int32_t max_sweeps;     /* Jacobi sweep cap; 0 selects 40 */
  int32_t profile;        /* 1: record per-phase clock ticks (tnrg_status) */
  const uint8_t *zz_mask; /* host [N-1]: bond carries the control u^zz */
  const uint8_t *xt_mask; /* host [N-1]: bond carries the crosstalk J */
  int32_t split_order;    /* 2 (or 0): U_l = R Z R; 1: U_l = X Y Z (Sec. II Eq. 4) */
  int32_t xt_model;       /* crosstalk (Sec. III Eq. 9): 0 = J Z Z (J is [.][N-1]);
                             1 = J^x XX + J^y YY + J^z ZZ (J is [.][N-1][3] holding
                             (J^x, J^y, J^z)); the two-site layer is then the
                             product of the bond exponentials in sweep order */
} tnrg_model;

/*
 * A batch of MPS in device memory, one per trajectory, in a fixed-capacity
 * layout.  Bond b (b = 0..N) has capacity cap_b = min(dcap, 2^b, 2^(N-b));
 * site j stores a (D_j, 2, D_{j+1}) tensor inside a (cap_j, 2, cap_{j+1})
 * row-major block: element (a, s, c) at
 *     data[t * tnrg_mps_traj_elems(N, dcap) + tnrg_mps_site_offset(N, dcap, j)
 *          + (a * 2 + s) * cap_{j+1} + c].
 * bond_dim[t][b] = D_b with D_0 = D_N = 1.
 */
typedef struct {
  int32_t n_traj;
  int32_t n_sites;
  int32_t dcap;
  int32_t *bond_dim; /* device [n_traj][n_sites + 1] */
  tnrg_c128 *data;   /* device [n_traj][tnrg_mps_traj_elems(n_sites, dcap)] */
} tnrg_mps_batch;

int32_t tnrg_bond_cap(int32_t n_sites, int32_t dcap, int32_t bond);
int64_t tnrg_mps_site_offset(int32_t n_sites, int32_t dcap, int32_t site);
int64_t tnrg_mps_traj_elems(int32_t n_sites, int32_t dcap);

/*
 * mps_evolve -- apply slices l_begin..l_end-1 of the time grid (Sec. II,
 * Eq. 4, second order; TEBD with SVD truncation) to every MPS of psi, in
 * place.  adjoint = 0: psi <- U_{l_end-1} ... U_{l_begin} psi, the two-site
 * sweep of slice l going left to right when M - 1 - l is odd (with
 * xt_model = 1 the bond visited first acts first).  adjoint = 1:
 * psi <- U_{l_begin}^dag ... U_{l_end-1}^dag psi, the sweep of slice l going
 * left to right when M - 1 - l is even, the exact adjoint of slice l.  The MPS entering a left-to-right
 * sweep must have its orthogonality centre on site 0 (sites 1..N-1
 * right-isometric), and on site N-1 for a right-to-left sweep; product states
 * qualify for both.
 *   ux, uy, uzz: device controls [M][N], [M][N], [M][N-1].
 *   J: device [psi->n_traj][N-1] (xt_model 0) or [psi->n_traj][N-1][3]
 *      (xt_model 1), the crosstalk of each trajectory.
 *   ws: device workspace of at least mps_evolve_workspace_bytes() bytes.
 */
size_t mps_evolve_workspace_bytes(const tnrg_model *md, int32_t n_traj,
                                  int32_t dcap);
int mps_evolve(const tnrg_model *md, const double *ux, const double *uy,
               const double *uzz, const double *J, int32_t l_begin,
               int32_t l_end, int32_t adjoint, const tnrg_mps_batch *psi,
               void *ws, size_t ws_bytes, tnrg_stream stream);

/*
 * mps_overlap -- out[t] = <bra_{t % bra->n_traj} | ket_t> by left transfer
 * matrices (Sec. II, Eq. 7 overlap).  bra->n_traj must divide ket->n_traj.
 * out is device [ket->n_traj].
 */
/* dcap: the larger of the two batches' capacities. */
size_t mps_overlap_workspace_bytes(int32_t n_traj, int32_t n_sites,
                                   int32_t dcap);
int mps_overlap(const tnrg_mps_batch *bra, const tnrg_mps_batch *ket,
                tnrg_c128 *out, void *ws, size_t ws_bytes, tnrg_stream stream);

/*
 * grape_fidelity_grad -- ensemble fidelity and its gradient with respect to
 * every control amplitude (Sec. II, Eq. 7; App. A), for K crosstalk samples
 * times R inputs, in one persistent launch with one workgroup per
 * trajectory.  Forward states are checkpointed every ckpt_stride slices
 * (0 selects ceil(sqrt(M))) and recomputed segment by segment during the
 * adjoint sweep.  With xt_model = 1 the u^zz derivative of bond b is taken
 * inside the sweep, between the forward state just after bond b and the
 * backward state just before it (App. A for the ordered bond product); the
 * adjoint then also re-runs each forward slice once to recover the forward
 * states inside it, and the workspace holds one more MPS.
 *   J: device [K][N-1] (xt_model 0) or [K][N-1][3] (xt_model 1).
 *   inputs: R MPS (each canonical with centre on site 0; product states are).
 *   targets: R MPS, right-canonical with unit norm (sites 1..N-1
 *            right-isometric).
 *   dcap: capacity of the internal states (bond dimensions above it raise
 *         TNRG_FLAG_OVERFLOW); 0 selects min(chi, 2^(N/2)); at most 128
 *         (TNRG_EUNSUPPORTED above).  Up to 32 the per-trajectory working
 *         buffers of a bond update live in LDS; above 32 in a per-trajectory
 *         region of the workspace (slower, for the rare large-bond cases).
 * Outputs (device): F[1]; g_ux[M][N], g_uy[M][N], g_uzz[M][N-1] (zero on
 * bonds without u^zz); overlaps[K*R] (may be NULL); traj_dO (may be NULL):
 * [K*R][2*M*N + M*(N-1)] complex dO/du per trajectory in the order ux, uy, uzz.
 */
size_t grape_workspace_bytes(const tnrg_model *md, int32_t K, int32_t R,
                             int32_t dcap, int32_t ckpt_stride);
int grape_fidelity_grad(const tnrg_model *md, const double *ux,
                        const double *uy, const double *uzz, int32_t K,
                        const double *J, int32_t R,
                        const tnrg_mps_batch *inputs,
                        const tnrg_mps_batch *targets, int32_t dcap,
                        int32_t ckpt_stride, double *F, double *g_ux,
                        double *g_uy, double *g_uzz, tnrg_c128 *overlaps,
                        tnrg_c128 *traj_dO, void *ws, size_t ws_bytes,
                        tnrg_stream stream);

/*
 * grape_forward / grape_backward -- the two halves of grape_fidelity_grad,
 * for callers that need the fidelity without the gradient (line searches,
 * finite differences) or that run the adjoint later, as the backward pass of
 * an autograd graph.  The arguments mean what they mean for
 * grape_fidelity_grad.
 *   grape_forward: the forward propagation (Sec. II, Eq. 4) of every
 *     trajectory, with the checkpoints every ckpt_stride slices kept in ws,
 *     then F[1] and overlaps[K*R] (may be NULL).  About a third of the work
 *     of grape_fidelity_grad.
 *   grape_backward: the adjoint sweep (App. A) from the checkpoints a
 *     grape_forward call left in ws; writes g_ux, g_uy, g_uzz and traj_dO
 *     (may be NULL).  All arguments, and the contents of the control, J,
 *     input and target buffers, must be those of that forward call; the
 *     forward call leaves a fingerprint of the sizes, the model and the
 *     buffer addresses in ws, and a backward call whose fingerprint differs
 *     sets TNRG_FLAG_STALE (tnrg_status returns TNRG_ESTALE) and computes
 *     nothing.  Values changed in place are not detected.  A grape_backward
 *     call leaves ws valid for another grape_backward.
 * The flags and counters read by tnrg_status after grape_backward cover both
 * calls.
 */
int grape_forward(const tnrg_model *md, const double *ux, const double *uy,
                  const double *uzz, int32_t K, const double *J, int32_t R,
                  const tnrg_mps_batch *inputs, const tnrg_mps_batch *targets,
                  int32_t dcap, int32_t ckpt_stride, double *F,
                  tnrg_c128 *overlaps, void *ws, size_t ws_bytes,
                  tnrg_stream stream);
int grape_backward(const tnrg_model *md, const double *ux, const double *uy,
                   const double *uzz, int32_t K, const double *J, int32_t R,
                   const tnrg_mps_batch *inputs, const tnrg_mps_batch *targets,
                   int32_t dcap, int32_t ckpt_stride, double *g_ux,
                   double *g_uy, double *g_uzz, tnrg_c128 *traj_dO, void *ws,
                   size_t ws_bytes, tnrg_stream stream);

/*
 * tnrg_status -- synchronise `stream`, then read the per-trajectory device
 * flags that the last call on `ws` left (n_traj entries).  Copies them to
 * host_flags when non-NULL; returns TNRG_OK, or the error of the most
 * severe flag (OVERFLOW, NOCONV, NONFINITE, STALE in that order).  stats (may be NULL)
 * receives 18 counts over all trajectories: {max bond dimension reached, max
 * Jacobi sweeps of one SVD, total Jacobi sweeps, number of SVDs, Jacobi flops
 * (36 m n(n-1)/2 per sweep of an m x n matrix), contraction flops (two-site
 * products, projections and transfer environments, 8 per complex
 * multiply-add)}, then, when the model's profile flag was set, clock ticks
 * of a 100 MHz counter summed over workgroups for the phases {site load,
 * theta, LQ preconditioner, Jacobi, split finish, left environments, right
 * environments and insertions, whole kernel}, then {Jacobi rounds, LQ
 * preconditioner steps}, then the clock ticks of {Jacobi rounds, Jacobi
 * end-of-sweep work}.
 */
int tnrg_status(const void *ws, int32_t n_traj, int32_t *host_flags,
                int64_t *stats, tnrg_stream stream);

/*
 * Launch plan (process-wide): the workgroup size used for internal states of
 * capacity dcap, one of 64, 128 or 256 threads (1, 2 or 4 waves per
 * trajectory), or 512 for capacities above 32 (TNRG_EINVAL otherwise); 0
 * restores the built-in choice.  Results do not depend on it
 * beyond rounding.  The autotuner of the Python binding times the choices on
 * the caller's workload and stores the fastest here.
 */
int tnrg_plan_set_threads(int32_t dcap, int32_t threads);
int32_t tnrg_plan_threads(int32_t dcap);

/*
 * Launch plan (process-wide) for capacities above 32: the one-sided Jacobi
 * SVD of a bond update (Sec. II, the truncated SVD) runs on a copy of its
 * matrix in LDS when it fits (about 150 KB: at most 72 columns of 128 rows),
 * which then leaves room for one workgroup per CU.  mode -1 (default) or 1:
 * on; 0: off (the matrix stays in the workspace and several workgroups
 * share a CU).  Results are bitwise the same either way.  TNRG_EINVAL for
 * other modes.
 */
int tnrg_plan_set_jacobi_lds(int32_t mode);

/*
 * Serving runtime: a request loop that runs fidelity+gradient evaluations of
 * concurrent optimisations (different N, chi, M, K, R) on one GPU with
 * continuous batching.  Each request is one persistent grape_fidelity_grad
 * launch; requests are admitted in arrival order as soon as a stream slot
 * and a block of the caller's device arena large enough for the request's
 * workspace are free, so requests that arrive while others run start at once
 * and their kernels share the GPU.  A request that was passed over because
 * its workspace did not fit is bypassed by at most max_bypass later ones.
 * The capacity bucket of each request is searched like the Python binding
 * does (4, 8, 16, 32, 64, 128 below min(chi, 2^(N/2)), then that value),
 * starting from the last bucket that worked for the same (N, M, chi, K, R)
 * in any server of the process;
 * a request whose bonds outgrow its bucket is requeued at the head with the
 * next one.
 *
 * Ownership: the arena (device memory) belongs to the caller and must
 * outlive the server; the server sub-allocates workspaces from it and
 * allocates no device memory itself (it creates its streams and events and
 * a pinned host buffer per stream for the device flags).  Every buffer a
 * request points to (controls, J, inputs, targets, outputs) must stay valid
 * until its completion has been returned.  The model and batch descriptors
 * are copied at submission.  One host thread drives a server.
 */
typedef struct tnrg_server tnrg_server;

typedef struct {
  const tnrg_model *md;
  const double *ux, *uy, *uzz; /* device controls [M][N], [M][N], [M][N-1] */
  int32_t K;
  const double *J; /* device [K][N-1] */
  int32_t R;
  const tnrg_mps_batch *inputs, *targets;
  int32_t dcap;    /* 0: bucket search */
  double *F;       /* device [1] */
  double *g_ux, *g_uy, *g_uzz;
  tnrg_c128 *overlaps; /* device [K*R] or NULL */
} tnrg_request;

typedef struct {
  int64_t ticket;
  int32_t status;   /* TNRG_OK or the error of the request */
  int32_t dcap;     /* capacity bucket of the last launch */
  int32_t launches; /* 1 + bucket regrowths */
  int32_t reserved;
  double queue_ms;  /* submission to first admission */
  double total_ms;  /* submission to completion seen by progress */
} tnrg_completion;

typedef struct {
  int32_t queued, running;
  int64_t submitted, admitted, completed, regrown, cancelled;
  size_t arena_bytes, arena_free, arena_largest_free;
} tnrg_server_info;

/* n_streams in 1..16; max_bypass >= 0; max_dcap: the largest capacity bucket
 * a request may grow to (0: no limit); a request whose bonds need more
 * completes with TNRG_EUNSUPPORTED (a service-level bound on the slow
 * global-scratch capacities above 32). */
int tnrg_server_create(void *arena, size_t arena_bytes, int32_t n_streams,
                       int32_t max_bypass, int32_t max_dcap,
                       tnrg_server **out);
/* Validates and queues a request; *ticket identifies its completion.  Does
 * not launch: tnrg_server_progress does.  Without a fixed req->dcap the
 * capacity buckets tried start at the larger of the input and target batch
 * capacities (the states hold those MPS before their first truncation). */
int tnrg_server_submit(tnrg_server *s, const tnrg_request *req,
                       int64_t *ticket);
/* Non-blocking step of the loop: collects finished launches (regrowing
 * buckets where needed), admits queued requests, and returns up to max_done
 * completions in done[0..*n_done-1] (the rest wait for the next call). */
int tnrg_server_progress(tnrg_server *s, tnrg_completion *done,
                         int32_t max_done, int32_t *n_done);
/* Drops every queued request that has not been admitted; their tickets go
 * to tickets[0..*n-1] (up to max). */
int tnrg_server_cancel_queued(tnrg_server *s, int64_t *tickets, int32_t max,
                              int32_t *n);
int tnrg_server_info_get(const tnrg_server *s, tnrg_server_info *info);
/* Waits for the running launches, then frees the server. */
int tnrg_server_destroy(tnrg_server *s);

/* Thread-local description of the last non-OK return. */
const char *tnrg_last_error(void);

/* Library version string. */
const char *tnrg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TNRG_H */
