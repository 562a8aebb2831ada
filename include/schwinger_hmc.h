/*
 * schwinger_hmc.h -- C ABI of the MI355X (gfx950) library for the hot path of the HMC
 * of the two-flavour lattice Schwinger model with (adapted) nested force-gradient
 * integrators (Shcherbakov, Ehrhardt, Finkenrath, Guenther, Knechtli, Peardon,
 * arXiv:1512.03812).
 *
 * Model (Sec. 3): an Lx x Lt lattice with U(1) links U_mu(n) = exp(i q_mu(n)), real
 * momenta p_mu(n), H = 1/2 sum p^2 + S_G + S_F (Eq. (12)), Wilson gauge action S_G
 * (Eq. (13)), pseudofermion action S_F = phi^dagger (D^dagger D)^{-1} phi (Eq. (14))
 * with the two-component Wilson-Dirac operator D of Sec. 3.  Gauge field periodic;
 * fermions periodic in x and antiperiodic in t (the paper leaves the boundary
 * conditions open; this library fixes that reading).
 *
 * Memory and ownership
 *   - The library never allocates device memory.  The caller allocates one device
 *     workspace of hmc_workspace_bytes() bytes (e.g. a torch tensor) and binds it with
 *     hmc_bind(); every field of the context lives inside it.  All other device
 *     pointers passed in are owned by the caller and are never freed.
 *   - All device work is enqueued on the HIP stream given to hmc_bind() (NULL = the
 *     default stream).  Calls that return per-chain info structs synchronise that
 *     stream before returning; the others return as soon as the work is enqueued.
 *   - The only host allocations are the context itself and a small pinned staging
 *     buffer for scalar read-backs (hipHostMalloc), both released by hmc_destroy().
 *
 * Native field layout (device pointers; see hmc_field / hmc_pack_*):
 *   A context holds n_chains independent lattices in one flat site space of V_total
 *   sites; chain c owns sites [offset_c, offset_c + Lx_c*Lt_c).  Inside a chain sites
 *   are ordered by parity (x+t)&1, then t, then x/2 (even-odd / checkerboard order).
 *   real link field (q, p, forces): double[2][V_total]          (mu = 0 is x, 1 is t)
 *   spinor field                  : double[2][V_total][2]       (spin s, then re/im)
 *   The lexicographic layout used by hmc_pack_* / hmc_unpack_* is, per chain,
 *   links double[Lt][Lx][2] (index 2n+mu, n = x + Lx t) and spinors
 *   double[Lt][Lx][2][2] (index 2n+s, then re/im), chains concatenated in order.
 *
 * Errors: every int-returning call returns HMC_OK (0) or a negative code; the text of
 * the last error is available from hmc_last_error().  A NULL context gives HMC_E_INVAL.
 */
#ifndef SCHWINGER_HMC_H
#define SCHWINGER_HMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HMC_OK = 0,
    HMC_E_INVAL = -1,   /* invalid argument (sizes, non-finite parameters, unbound context) */
    HMC_E_NOMEM = -2,   /* workspace too small */
    HMC_E_NOCONV = -3,  /* a CG solve hit max_iter before reaching its tolerance */
    HMC_E_HIP = -4,     /* a HIP runtime call failed */
    HMC_E_NAN = -5      /* a non-finite energy difference (the trajectory is rejected) */
};

/* Integrators of Sec. 2.2 */
enum {
    HMC_LEAPFROG = 0,          /* Eq. (3) */
    HMC_OMELYAN_5STAGE = 1,    /* Eq. (4): 5-stage scheme, lambda = 1/6 */
    HMC_FORCE_GRADIENT = 2,    /* Eq. (5), force-gradient term via the shifted force */
    HMC_NESTED_FG = 3,         /* Eq. (10) */
    HMC_ADAPTED_NESTED_FG = 4, /* Eq. (11) */
    HMC_NESTED_LEAPFROG = 5,   /* Eq. (8) */
    HMC_NESTED_5STAGE = 6,     /* Eq. (9) */
    HMC_OMELYAN_11STAGE = 7    /* Eq. (6), with the fourth-order sigma, eta, lambda, theta of
                                  Omelyan, Mryglod and Folk (2003), their Eq. (71) */
};

enum { HMC_PREC_FP64 = 0, HMC_PREC_MIXED = 1 };

/* which force for hmc_fg_shifted_force, hmc_hessian_vector and hmc_force_gradient_term */
enum { HMC_FORCE_GAUGE = 0, HMC_FORCE_FERMION = 1, HMC_FORCE_TOTAL = 2 };

/* How the integrators' force-gradient kicks e^{eps B - (h^3/72) C} are formed (Sec. 2.2):
 * HMC_FG_SHIFT (default): p -= eps F(q - (h^2/24) F(q)), the Taylor-expansion variant;
 * HMC_FG_EXACT: p -= eps F(q) - (h^3/72) C(q) with C of Eq. (19) from hmc_force_gradient_term. */
enum { HMC_FG_SHIFT = 0, HMC_FG_EXACT = 1 };

/* named fields inside the bound workspace (hmc_field) */
enum {
    HMC_FIELD_Q = 0,    /* link angles q, real link field (the state of the chains) */
    HMC_FIELD_P = 1,    /* momenta p, real link field */
    HMC_FIELD_PHI = 2,  /* pseudofermion phi of the current trajectory, spinor field */
    HMC_FIELD_CHI = 3,  /* chi = D xi after the last fermion force, spinor field (Eq. (18)) */
    HMC_FIELD_XI = 4,   /* xi = (D^dagger D)^{-1} phi after the last fermion force, spinor field */
    HMC_FIELD_F = 5,    /* last force field a trajectory stored, real link field (kicks that
                           involve the gauge force apply it directly and store none) */
    HMC_FIELD_ZETA = 6  /* Gaussian zeta of the last refresh (phi = D^dagger zeta), spinor field */
};

typedef struct hmc_ctx hmc_ctx;

/* per-chain result of a CG solve */
typedef struct {
    int iters;             /* CG iterations (FP32 iterations in mixed precision) */
    int converged;         /* 1 if the tolerance was reached */
    int reliable_updates;  /* FP64 residual recomputations (mixed precision), else 0 */
    int pad;
    double rel_resid;      /* ||r|| / ||phi|| of the solver's own residual */
    double rel_resid_true; /* ||phi - D^dagger D x|| / ||phi|| recomputed in FP64 */
} hmc_cg_info;

/* per-chain result of one HMC trajectory (Sec. 2.1) */
typedef struct {
    double dH;           /* H(U', P') - H(U, P), summed as per-term differences */
    double H0, H1;       /* Hamiltonian (Eq. (12)) before and after the molecular dynamics */
    double plaquette;    /* mean Re P(n) of the chain after the Metropolis step */
    double u;            /* Metropolis uniform */
    int accepted;        /* 1 if U' was accepted */
    int status;          /* HMC_OK, HMC_E_NOCONV or HMC_E_NAN for this chain */
    int n_force_evals;   /* fermion-force evaluations of the molecular dynamics */
    int n_solves;        /* CG solves actually run (repeated forces at unchanged links are reused) */
    int n_dinv;          /* inversions of D in the paper's count: 2 per fermion-force evaluation,
                            plus 2 per Hessian-vector solve of an exact force-gradient term */
    int pad;
    long long n_cg_iters;  /* total CG iterations of this chain over the trajectory */
} hmc_traj_info;

/* ---------------------------------------------------------------- set-up */

/* One Lx = Lt = L chain.  L even and >= 2; beta, m0 finite.  The Philox key is seed;
 * the chain index (counter word 3) is 0.  Links start cold (q = 0). */
int hmc_init(hmc_ctx **out, int L, double beta, double m0, uint64_t seed);

/* One Lx x Lt chain (both even, >= 2). */
int hmc_init_ex(hmc_ctx **out, int Lx, int Lt, double beta, double m0, uint64_t seed);

/* n_chains independent chains (chain c uses Philox chain index c). */
int hmc_batch_init(hmc_ctx **out, int n_chains, const int *Lx, const int *Lt, const double *beta,
                   const double *m0, uint64_t seed);

/* Device bytes the caller must provide to hmc_bind(). */
size_t hmc_workspace_bytes(const hmc_ctx *ctx);

/* Binds the caller-owned device workspace (>= hmc_workspace_bytes, 256-byte aligned)
 * and the HIP stream (hipStream_t passed as void*).  Must precede every device call;
 * may be called again to move the context to another workspace/stream (fields are
 * not copied). */
int hmc_bind(hmc_ctx *ctx, void *dev_workspace, size_t bytes, void *hip_stream);

/* Device pointer (and size in bytes) of a named field inside the workspace.  The library
 * keeps the complex links U = exp(i q) and solver results derived from q between calls;
 * every hmc_field call, and every library call that changes q, invalidates them.  A caller
 * that writes q through a pointer obtained earlier calls hmc_mark_links_changed first. */
int hmc_field(hmc_ctx *ctx, int which, void **dev_ptr, size_t *bytes);
int hmc_mark_links_changed(hmc_ctx *ctx);

/* n_chains, V_total, and per chain (arrays of n_chains, any may be NULL) the flat
 * offset and extents. */
int hmc_geometry(const hmc_ctx *ctx, int *n_chains, long long *v_total, int *offsets, int *Lx,
                 int *Lt);

/* Layout conversion between the lexicographic and the native layout (device pointers,
 * the two buffers must not overlap). */
int hmc_pack_links(hmc_ctx *ctx, const double *lexico, double *native);
int hmc_unpack_links(hmc_ctx *ctx, const double *native, double *lexico);
int hmc_pack_spinor(hmc_ctx *ctx, const double *lexico, double *native);
int hmc_unpack_spinor(hmc_ctx *ctx, const double *native, double *lexico);

/* Links: q = 0 (cold) or q uniform in [-pi, pi) from Philox stream 0 (hot start). */
int hmc_cold_start(hmc_ctx *ctx);
int hmc_hot_start(hmc_ctx *ctx);

/* Trajectory counter used as Philox counter word 2 by the next hmc_trajectory
 * (starts at 0, incremented by every trajectory; set it to resume a chain). */
int hmc_set_trajectory_counter(hmc_ctx *ctx, uint32_t traj);
uint32_t hmc_get_trajectory_counter(const hmc_ctx *ctx);

/* Solver tolerance and iteration cap used inside hmc_trajectory (default 1e-12, 100000).
 * reliable_delta: in mixed precision, the FP64 residual is recomputed whenever the
 * FP32 residual has dropped by this factor (default 1e-4). */
int hmc_set_solver(hmc_ctx *ctx, double tol, int max_iter, double reliable_delta);

/* Drop the fermion action (pure-gauge HMC; used to check the gauge part against the exact
 * plaquette of 2-D U(1)).  Default 0. */
int hmc_set_quenched(hmc_ctx *ctx, int quenched);

/* Every `every` CG iterations the host reads back how many chains have converged
 * (default 32; the interval doubles up to 4 times that while no chain converges).  Iterations
 * launched after a chain converged do no work for it. */
int hmc_set_check_interval(hmc_ctx *ctx, int every);

/* Chains with at most vmax sites solve their CG inside one persistent workgroup (the
 * search direction and D p held in LDS), concurrently with the multi-workgroup kernels that
 * handle the larger chains; 0 disables it.  Default and maximum 2048. */
int hmc_set_persistent_limit(hmc_ctx *ctx, int vmax);

/* Chain groups (Sec. 2.1: the chains are independent HMC updates).  With groups > 1,
 * hmc_trajectory splits the chains into that many contiguous ranges of about equal sites and
 * advances each range through the whole trajectory (refresh, molecular dynamics with its own
 * solves, convergence checks and workgroup compaction, energies, Metropolis) on its own
 * stream, driven by its own host thread (the first range on the calling thread and the bound
 * stream; the others on library-owned streams, after the work already on the bound stream,
 * which waits for all of them before the call returns).  One range's kernels then fill the
 * GPU while another's host waits at a convergence check or its solve drains.  Each chain's
 * arithmetic is the same either way: results are bit-identical for any group count.  With
 * more groups than chains each chain is a group.  Other calls (hmc_cg_solve, hmc_integrate,
 * whole-trajectory graphs of hmc_set_graph) run the chains as one set.  The kernel statistics
 * of hmc_get_kernel_stats add up the groups' launches (which overlap in time).  groups: 1..4,
 * default 1. */
int hmc_set_cg_groups(hmc_ctx *ctx, int groups);

/* CG kernels of the multi-workgroup solver (Sec. 3 calls the solve "D^-1").  With on = 1
 * a solve runs one fused kernel per CG iteration when every chain it iterates lets a
 * workgroup own whole lattice rows (block/2 a multiple of Lx/2 with Lt at least 4 rows
 * more than a workgroup owns, or the whole chain within one workgroup) and the LDS windows
 * fit: the recurrences are regrouped so that one reduction point per iteration suffices
 * (the squared residual norm that sets beta is predicted from <r, A p> and ||A p||^2), and
 * the stencil rows two beyond a workgroup's own are recomputed.  Otherwise, or with on = 0
 * (default), each iteration takes two kernels.  Both give the CG iterates up to rounding.
 * The fused kernel moves 18 % fewer bytes per iteration and saves a kernel boundary, but
 * the recomputed rows and its register use make it slower on MI355X (about 15 % on the
 * batched workload), so it runs only when asked for. */
int hmc_set_fused_cg(hmc_ctx *ctx, int on);

/* Threads per workgroup of the site kernels (128..1024, multiple of 64; default 256). */
int hmc_set_block_size(hmc_ctx *ctx, int block);

/* Variants of the two CG step kernels (compile-time instantiations):
 * HMC_STEP_PLAIN     one lattice site per thread (default);
 * HMC_STEP_TWO_SITES two sites per thread (a workgroup's strip of each parity plane is twice
 *                    as long, so fewer of its stencil neighbours lie outside it);
 * HMC_STEP_RESIDENT  a grid of at most the workgroups resident on the GPU at once walks the
 *                    workgroup list (no partly filled last round, fewer workgroup starts);
 * HMC_STEP_WAVES8    at most 64 VGPRs per thread, so 8 waves per SIMD fit.
 * All give the same iterates.  The tables are rebuilt for the variant's sites per thread. */
enum { HMC_STEP_PLAIN = 0, HMC_STEP_TWO_SITES = 1, HMC_STEP_RESIDENT = 2, HMC_STEP_WAVES8 = 3 };
int hmc_set_step_variant(hmc_ctx *ctx, int variant);

/* A trajectory schedule for the autotuner's chain-group search. */
typedef struct {
    int scheme, n_outer, n_inner, pad;
    double tau;
} hmc_tune_schedule;

/* The autotuner's pick (and what it cost to find). */
typedef struct {
    int block;             /* workgroup size of the site kernels */
    int persistent_limit;  /* persistent-solver limit (sites) */
    int step_variant;      /* HMC_STEP_* */
    int check_interval;    /* CG slots between convergence checks */
    int groups;            /* chain groups (hmc_set_cg_groups) */
    int candidates;        /* configurations timed */
    double reliable_delta; /* mixed precision: reliable-update factor */
    double solve_ms;       /* mean wall time of one solve with the pick */
    double traj_ms;        /* wall time of one trajectory with the pick (0: groups not searched) */
} hmc_tune_info;

/* Autotuner: times CG solves of this context's own chains at its current links (with a
 * fresh pseudofermion: p and phi are overwritten; q is kept) and keeps the fastest setting,
 * one dimension after the other: workgroup size {128, 256, 512, 1024} x persistent-solver
 * limit {0, 1024, 2048 where chains fit}; step-kernel variant (sites per thread 1 or 2,
 * resident grid, 64-VGPR bound); convergence-check interval {16, 32, 64}; in mixed
 * precision the reliable-update factor {1e-3, 1e-4, 1e-5} (which changes the iterates within
 * the tolerance).  If traj is not NULL and the context has several chains, it then times one
 * trajectories of that schedule (the mean of two, after a warm-up one) for 1..4 chain groups and keeps
 * the fastest; q and the trajectory counter are restored afterwards.  tol: the solver
 * tolerance of the timed solves and trajectories. */
int hmc_autotune(hmc_ctx *ctx, int prec, double tol, const hmc_tune_schedule *traj,
                 hmc_tune_info *out);

/* ---------------------------------------------------------------- operators (Sec. 3) */

/* out = D in: (D psi)(n) = (2+m0) psi(n) - 1/2 sum_mu [(1 - sigma_mu) U_mu(n) psi(n+mu)
 * + (1 + sigma_mu) U_mu^dagger(n-mu) psi(n-mu)], links from the context's q.
 * in/out: native spinor fields (device), must not overlap. */
int hmc_dslash(hmc_ctx *ctx, const void *in, void *out);

/* out = D^dagger in (the conjugate transpose of D above). */
int hmc_dslash_dagger(hmc_ctx *ctx, const void *in, void *out);

/* Solves D^dagger D x = phi for every chain by CG from x = 0 (the "D^{-1}" of Sec. 3:
 * one solve is two inversions of D).  Stops per chain when ||r|| <= tol ||phi||;
 * prec = HMC_PREC_MIXED runs the iterations in FP32 with FP64 reliable updates and
 * stops on the FP64 true residual.  info: array of n_chains (may be NULL).
 * Each chain stops on its own: a chain that reaches max_iter iterations, or whose residual
 * norm is not finite (a NaN or Inf in its links or phi), stops unconverged with x holding its
 * last iterate, while the other chains go on; info[c].converged tells them apart.  Returns
 * HMC_E_NAN if some chain's residual was not finite, else HMC_E_NOCONV if some chain hit
 * max_iter, else HMC_OK. */
int hmc_cg_solve(hmc_ctx *ctx, const void *phi, void *x, double tol, int max_iter, int prec,
                 hmc_cg_info *info);

/* hmc_cg_solve in FP64 that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): every chain's CG runs in the one-workgroup persistent solver, and all kernel
 * scratch (the links U = exp(i q), the CG states, the chain list, the true-residual
 * intermediate and its partial sums) lives in one static device array of the library
 * (4.5 MiB, held by each GPU the library runs on until the process ends) instead of the
 * bound workspace.  The call makes no hipMalloc, hipFree or other allocating call; it reads
 * q and the chain tables from the bound workspace and writes only x and info.
 * Limits: V_total <= 65536 sites, n_chains <= 1024, every chain at most 2048 sites
 * (HMC_E_NOMEM / HMC_E_INVAL with a message otherwise).  Results are those of hmc_cg_solve
 * with prec = HMC_PREC_FP64 on the same context, bit for bit; return codes as there.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU (from
 * several streams or threads) race and must be serialised by the caller.  The current device
 * must be the one the context was bound on. */
int hmc_cg_solve_noalloc(hmc_ctx *ctx, const void *phi, void *x, double tol, int max_iter,
                         hmc_cg_info *info);

/* ---------------------------------------------------------------- forces (Sec. 3) */

/* f = dS_F/dq (Eqs. (17), (18)): solves xi = (D^dagger D)^{-1} phi, forms chi = D xi and
 * evaluates the fermion force into the real link field f (device, caller-owned).
 * chi and xi stay in the workspace (HMC_FIELD_CHI / HMC_FIELD_XI).  sf (n_chains
 * doubles, host, may be NULL) receives S_F = Re phi^dagger xi per chain.  f may be NULL:
 * then only xi, chi and S_F are formed (the forward pass of an adjoint-force pair). */
int hmc_fermion_force(hmc_ctx *ctx, const void *phi, double *f, double tol, int max_iter, int prec,
                      hmc_cg_info *info, double *sf);

/* The force kernel alone: f from given chi, xi (the adjoint of S_F, Eq. (17)). */
int hmc_fermion_force_chixi(hmc_ctx *ctx, const void *chi, const void *xi, double *f);

/* F = dS_G/dq + dS_F/dq (Eq. (15)) with the fermion part from given chi, xi: the adjoint
 * of S = S_G + S_F, used as the backward pass of an autograd function. */
int hmc_total_force_chixi(hmc_ctx *ctx, const void *chi, const void *xi, double *F);

/* g = dS_G/dq = beta Im(P_{mu nu}(n) - P_{mu nu}(n - nu)), Eq. (16), from the context's q. */
int hmc_gauge_force(hmc_ctx *ctx, double *g);

/* Actions per chain (host arrays of n_chains, any may be NULL): S_G (Eq. (13)), mean
 * plaquette, and, if phi is not NULL, S_F = phi^dagger (D^dagger D)^{-1} phi (Eq. (14))
 * solved to tol in FP64.  If a chain's solve stops unconverged, S_G and the plaquette are still
 * filled, that chain's S_F is NaN and the call returns HMC_E_NOCONV (iteration cap) or
 * HMC_E_NAN (non-finite residual). */
int hmc_actions(hmc_ctx *ctx, const void *phi, double tol, double *s_gauge, double *plaquette,
                double *s_fermion);

/* ---------------------------------------------------------------- updates (Sec. 2.1) */

/* e^{eps A}: q += eps p (U' = exp(i p eps) U) on the context's fields. */
int hmc_update_links(hmc_ctx *ctx, double eps);

/* e^{eps B}: p -= eps F, F a real link field (device). */
int hmc_update_momenta(hmc_ctx *ctx, double eps, const double *F);

/* Force at the force-gradient-shifted links: F_out = F(q + c_h2 F(q)) with F the gauge,
 * fermion or total force (which = HMC_FORCE_*); c_h2 = -h^2/24 gives the Taylor form of
 * the force-gradient kick (Sec. 2.2).  q itself is left unchanged.  phi is needed unless
 * which == HMC_FORCE_GAUGE.  info: n_chains entries for the last solve (may be NULL). */
int hmc_fg_shifted_force(hmc_ctx *ctx, double c_h2, int which, const void *phi, double *F_out,
                         int prec, hmc_cg_info *info);

/* Hessian-vector product out = H v, H the matrix of second derivatives d^2 S / dq_a dq_b of
 * S = S_G (which = HMC_FORCE_GAUGE), S_F (FERMION) or S_G + S_F (TOTAL) at the context's
 * links, v and out real link fields (device, native layout, out may not alias v).  For the
 * fermion part (Sec. 3, Eqs. (21)-(23)) xi = (D^dagger D)^{-1} phi and chi = D xi are
 * solved for first (left in HMC_FIELD_XI/CHI), then one more solve of D^dagger D gives the
 * Z_2 of Eq. (23) for the weight v (Z_1 follows as D Z_2 - dD[v] xi).  phi is needed unless
 * which == HMC_FORCE_GAUGE.  Solver tolerance and iteration cap are those of
 * hmc_set_solver.  info: n_chains entries for the Hessian solve (may be NULL).  Returns
 * HMC_E_NOCONV if a solve did not converge (out is then inaccurate). */
int hmc_hessian_vector(hmc_ctx *ctx, int which, const void *phi, const double *v, double *out,
                       int prec, hmc_cg_info *info);

/* The force-gradient term C = 2 H F = grad |F|^2 of Eq. (19) for the force set which:
 * C_GG (GAUGE), C_FF (FERMION, the part the nested schemes use), or
 * C_GG + C_FG + C_GF + C_FF (TOTAL) of Eq. (20).  Two solves of D^dagger D when the fermion
 * part is included (force, then the Hessian solve).  C: real link field (device).  info:
 * n_chains entries for the Hessian solve (may be NULL). */
int hmc_force_gradient_term(hmc_ctx *ctx, int which, const void *phi, double *C, int prec,
                            hmc_cg_info *info);

/* Selects HMC_FG_SHIFT or HMC_FG_EXACT for the force-gradient kicks of hmc_trajectory and
 * hmc_integrate (schemes HMC_FORCE_GRADIENT, HMC_NESTED_FG, HMC_ADAPTED_NESTED_FG). */
int hmc_set_fg_mode(hmc_ctx *ctx, int mode);

/* ---------------------------------------------------------------- HMC (Sec. 2.1, 2.2) */

/* One HMC trajectory for every chain: momentum and pseudofermion refresh from Philox
 * streams 1 and 2 (phi = D^dagger zeta), molecular dynamics with the given scheme
 * (h = tau / n_outer; n_inner = M inner steps per inner call of the nested schemes,
 * ignored otherwise), Delta H in FP64, Metropolis test with stream 3, links restored on
 * rejection.  info: n_chains entries (may be NULL).  A chain fails when one of its solves
 * stops unconverged (status HMC_E_NOCONV at the iteration cap of hmc_set_solver,
 * HMC_E_NAN on a non-finite residual) or its Delta H is not finite (HMC_E_NAN); a failing
 * chain is rejected and gets its links back, and every other chain computes exactly what it
 * computes without the failing one.  Returns HMC_OK, or the first failing chain's status. */
int hmc_trajectory(hmc_ctx *ctx, int scheme, double tau, int n_outer, int n_inner, int prec,
                   hmc_traj_info *info);

/* hmc_trajectory on n (1..8) contexts at once, one host thread each (the calling thread
 * takes ctxs[0]).  Every context must be bound, each to a stream of its own; their work
 * overlaps on the GPU, so that one context's kernels fill the gaps of another (its host
 * waits at convergence checks, the tail of its solves).  Each context computes exactly what
 * hmc_trajectory computes.  infos[k] (may be NULL, or NULL entries): n_chains entries of
 * context k; rcs[k] (may be NULL): its return code.  Returns the first nonzero code, or
 * HMC_E_INVAL for a repeated context or stream.  The calling thread's current HIP device is
 * the same on return as on entry. */
int hmc_trajectories_concurrent(hmc_ctx **ctxs, int n, int scheme, double tau, int n_outer,
                                int n_inner, int prec, hmc_traj_info **infos, int *rcs);

/* Captured trajectories.  With on != 0, hmc_trajectory runs from HIP graphs:
 *  - when every chain is within the persistent solver's limit, its whole device work (refresh,
 *    molecular dynamics with every solve, energies, Metropolis) is recorded as one graph on
 *    first use of a (scheme, tau, n_outer, n_inner, prec) schedule and replayed afterwards: one
 *    launch per trajectory and no host round trip until its results are read;
 *  - otherwise the iteration slots of every solve run as a captured chunk of check-interval
 *    slots (both CG step kernels per slot over the active workgroup list, whose length the
 *    kernels read from the device, then the compaction), replayed until the host, reading
 *    the active count once per chunk, finds every chain stopped; the rest of the trajectory
 *    is launched as usual.  This also holds inside chain groups (hmc_set_cg_groups).
 * The results are those of the eager path, bit for bit.  Any setter (solver, quenched,
 * force-gradient mode, persistent limit, workgroup size, step variant) and a new binding
 * discard the captured graphs.  Default off. */
int hmc_set_graph(hmc_ctx *ctx, int on);

/* The refresh of Sec. 2.1 alone, for the current trajectory counter (not incremented):
 * p ~ N(0,1) from Philox stream 1, zeta with density exp(-zeta^dagger zeta) from stream 2,
 * phi = D^dagger zeta at the current links (so S_F(U) = zeta^dagger zeta). */
int hmc_refresh(hmc_ctx *ctx);

/* Molecular dynamics only, from the context's q, p and phi (no refresh, no Metropolis). */
int hmc_integrate(hmc_ctx *ctx, int scheme, double tau, int n_outer, int n_inner, int prec,
                  hmc_traj_info *info);

/* ---------------------------------------------------------------- kernel timing */

/* Sampled event timing of the CG step kernels (which = 0: step 1, the x update and
 * t = D p, or the whole fused iteration; which = 1: step 2, r -= alpha D^dagger t).
 * While on, in every 32nd CG iteration slot (away from the host's convergence checks) each
 * kernel is launched with a start and an end HIP event that its own dispatch stamps, and
 * step 1 records on the device the algorithmic bytes of both steps for the chains it
 * iterates (their sites times the bytes per site of the slot's mode); the bytes are summed
 * beside the durations at the end of each solve.  hmc_set_timing resets the statistics. */
typedef struct {
    long long launches;       /* CG slots launched while timing was on */
    long long timed_launches; /* launches of this kernel bracketed by events */
    double timed_ms;          /* their summed event-measured duration */
    double timed_bytes;       /* their summed algorithmic bytes */
    int sample_every;         /* sampling period in slots */
    int fused;                /* 1: the solves ran the fused iteration, whose kernel is
                                 index 0 (index 1 then holds nothing) */
    double all_bytes;         /* algorithmic bytes of this kernel over every slot launched while
                                 timing was on (two-kernel iteration), timed or not */
} hmc_kernel_stat;

int hmc_set_timing(hmc_ctx *ctx, int on);
int hmc_get_kernel_stats(hmc_ctx *ctx, int which, hmc_kernel_stat *out);

/* Streaming copy dst = src of `bytes` bytes on the bound stream (device pointers, both
 * 16-byte aligned, bytes a multiple of 16; src and dst must not overlap): one 16-byte
 * nontemporal load and store per thread.  Not part of the method: it is the measured
 * bandwidth ceiling placed beside the roofline figures, and the kernel whose HBM byte
 * counters calibrate the counter readings of the others.  Returns HMC_E_INVAL for
 * misaligned or unbound arguments. */
int hmc_stream_copy(hmc_ctx *ctx, const void *src, void *dst, size_t bytes);

/* ---------------------------------------------------------------- misc */

const char *hmc_last_error(const hmc_ctx *ctx);
int hmc_destroy(hmc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SCHWINGER_HMC_H */
