// Host-side launchers of the HIP kernels (internal interface of the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace shmc {

// Geometry of a batch as the kernels see it.
struct Geo {
    const ChainInfo *chains;  // device, n_chains entries
    const BlockWork *work;    // device, nblocks entries (hardware order; may be a compacted list)
    int nblocks;              // workgroups launched
    int nlog;                 // logical workgroups of the whole batch (size of a partials row)
    int nchains;
    int Vtot;                 // sites of the flat site space (the stride between field planes)
    int block;                // threads per workgroup
    int site0, nsites;        // the contiguous flat-site range of these chains
};

// Per-chain CG state.  Double-buffered by the parity of the iteration slot: the first
// kernel of slot k reads state[(k+1)&1] and its chain-leading workgroup writes
// state[k&1]; the second kernel of slot k reads state[k&1].
struct CGState {
    double rho;     // ||r||^2 of the residual entering this slot
    double rho_p;   // ||r||^2 one CG iteration earlier (beta denominator after an update)
    double target;  // tol^2 ||phi||^2
    double phi2;    // ||phi||^2
    double rmax2;   // mixed: ||r||^2 at the last FP64 residual recomputation
    double beta;    // beta of this slot's direction update
    double delta2;  // mixed: reliable-update trigger factor squared
    double alpha;   // normal slot: this slot's alpha, whose x update the next slot applies;
                    // update slot: the alpha still owed to x, folded in by its step 2
    double t2;      // fused iteration: ||D p||^2 of the last direction (kept across an update)
    double s2;      // fused iteration: ||D^dagger D p||^2 of the last direction
    int iters;      // CG iterations completed
    int converged;  // 0 while iterating; kConverged once the stopping test passed; a chain
                    // that stops without converging holds kStopMaxIter (iteration cap) or
                    // kStopNonFinite (its residual norm is not finite)
    int mode;       // kModeInit, kModeNormal, kModeUpdate (this slot), kModeUpdate2
    int n_updates;  // mixed: FP64 residual recomputations completed
    int buf;        // fused iteration: which of the two buffers holds r, s and p
    int pad[3];
};
static_assert(sizeof(CGState) % 16 == 0, "CGState alignment");
// kModeUpdate2: the second half of a fused-iteration residual recomputation.
enum { kModeInit = 0, kModeNormal = 1, kModeUpdate = 2, kModeUpdate2 = 3 };
// CGState::converged: nonzero once a chain has stopped; only kConverged means converged.
enum { kConverged = 1, kStopMaxIter = 2, kStopNonFinite = 3 };

// Sampled slots per solve whose bytes the timing records (rows of the device byte table).
constexpr int kMaxSamples = 256;
// Algorithmic bytes per lattice site of the CG step kernels (each distinct input read once,
// each output written once; stencil neighbours come from cache).  Step 1 also applies the
// previous iteration's x update.
//   FP64 solver   step 1: r 32 + p_old 32 + U 32 + x 32 read, p 32 + t 32 + x 32 = 224
//                 step 2: t 32 + U 32 + r 32 read, r 32 written                  = 128
//   mixed, FP32   step 1: r 16 + p_old 16 + U 8 + x 16 read, p 16 + t 16 + x 16  = 104
//                 step 2: t 16 + U 8 + r 16 read, r 16 written                   =  56
//                 (U: the two FP32 link angles of the site)
//   mixed, FP64 residual recomputation
//                 step 1: x64 32 + x32 16 + p_old 16 + U64 32 read, t64 32 + p 16 = 144
//                 step 2: t64 32 + U64 32 + phi 32 + x64 32 + x32 16 + p 16 read,
//                         x64 32 + x32 16 + r32 16 written                      = 224
// (The first slot of a solve reads neither p_old nor x; it is counted like the others.)
constexpr double kBytesFp64Step1 = 224.0, kBytesFp64Step2 = 128.0;
constexpr double kBytesFp32Step1 = 104.0, kBytesFp32Step2 = 56.0;
constexpr double kBytesUpdateStep1 = 144.0, kBytesUpdateStep2 = 224.0;
// The fused iteration (one kernel per CG iteration):
//   normal slot, FP64  : r, s, p, x 4 x 32 + U 32 read, r, s, p, x 4 x 32 written = 288
//   normal slot, FP32  : r, s, p, x 4 x 16 + U 8 read, r, s, p, x 4 x 16 written  = 136
//   mixed, residual recomputation, first slot : x64 32 + x32 16 + U64 32 read,
//                                                t64 32 written                   = 112
//                                  second slot: t64 32 + U64 32 + phi 32 + x64 32 + x32 16
//                                                + s 16 read, x64 32 + x32 16 + r 16  = 224
constexpr double kBytesIterFp64 = 288.0, kBytesIterFp32 = 136.0;
constexpr double kBytesIterUpdate1 = 112.0, kBytesIterUpdate2 = 224.0;

// Partial sums: row k of partials holds one double per logical workgroup.
constexpr int kMaxReduce = 8;
// A consumer workgroup re-adds its chain's partials itself when the chain has at most this
// many workgroups; larger chains get their totals from a finalize kernel instead.
constexpr int kMaxChainBlocks = 2048;
// Slices of such a chain's partials that k_finalize_large sums separately (one workgroup
// each); the consumers re-add the slice sums.
constexpr int kFinSlices = 64;

// ---------------------------------------------------------------- layout
// to_native: nat <- lex, else lex <- nat
void launch_pack_links(const Geo &g, double *lex, double *nat, bool to_native, hipStream_t s);
void launch_pack_spinor(const Geo &g, double2 *lex, double2 *nat, bool to_native, hipStream_t s);

// ---------------------------------------------------------------- links
// U = exp(i q) with the antiperiodic sign on the t-links leaving the last time slice;
// A32 (may be null) receives the FP32 angles of the mixed-precision solver.
void launch_make_links(const Geo &g, const double *q, double2 *U64, float *A32, hipStream_t s);

// ---------------------------------------------------------------- Dirac operator
void launch_dslash64(const Geo &g, const double2 *U, const double2 *in, double2 *out, bool dagger,
                     hipStream_t s);

// ---------------------------------------------------------------- CG on D^dagger D
struct CGFields {
    const double2 *phi;       // FP64 right-hand side
    double2 *x64;             // FP64 solution (accumulated solution in mixed precision)
    double2 *r64, *t64;       // FP64 residual and D p (FP64 solver); t64 is also the mixed scratch
    float4 *x32, *r32, *t32;  // mixed: FP32 partial solution, residual, D p (one float4 per site)
    const double2 *U64;
    const float *A32;  // FP32 link angles [2][Vtot] (boundary sign folded in as +pi)
    double *p1, *p2;          // partial rows: ||D p||^2 (step 1) and ||r||^2 (step 2)
    double *fin1, *fin2;      // per-chain slice sums [nchains][kFinSlices] of p1, p2 for chains
                              // above kMaxChainBlocks
    CGState *st;              // [2][nchains]
    double *samples;          // timing: [kMaxSamples][nchains][2] bytes of sampled slots
    double *all_bytes;        // timing: [nchains][2] running sums of the bytes of every slot
    const int *active;        // step kernels: if set, the number of work entries is *active (the
                              // grid may be larger; the workgroups beyond it exit at once)
};
// Variants of the two CG step kernels (compile-time instantiations the autotuner chooses
// among): one site per thread (plain), two sites per thread (the workgroup tables must then
// be built with spt = 2), a resident grid that walks the workgroup list, and at most 64
// VGPRs (8 waves per SIMD).
enum { kStepPlain = 0, kStepTwoSites = 1, kStepResident = 2, kStepWaves8 = 3, kNumStepVariants = 4 };
int step_variant_spt(int variant);

// x = 0, r = phi, partial ||phi||^2 -> p2, state[1] = initial.
void launch_cg_init(const Geo &g, const CGFields &f, bool mixed, double delta, hipStream_t s);
// Slot k, first kernel: decide (converged / beta / reliable update) from the partials of
// the previous slot, apply the previous slot's x += alpha p_old, then p_new = r + beta p_old
// and t = D p_new with partial ||t||^2 (or, in a reliable-update slot,
// t64 = D (x64 + x32 + alpha p_old)).  decide_only: state update and the owed x update only.
// A chain stops unconverged once it has done max_iter iterations or its residual norm is
// not finite.  ev0/ev1 (optional): stamped with the kernel's own start and end (timing).
void launch_cg_step1(const Geo &g, const CGFields &f, bool mixed, int variant, int slot, double tol,
                     int max_iter, const void *p_old, void *p_new, bool decide_only, int sample,
                     hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// sums[2 b + k] = sum over chains of samples[b][chain][k], b < n; the rows are zeroed.
void launch_sample_sums(double *samples, int n, int nchains, double *sums, hipStream_t s);
// Slot k, second kernel: alpha from the partials of step 1 (kept in the state for the next
// slot's x update), r -= alpha D^dagger t with partial ||r||^2 (or the FP64 residual
// recomputation, which also folds x32 and the owed alpha p into x64).
void launch_cg_step2(const Geo &g, const CGFields &f, bool mixed, int variant, int slot,
                     const void *p_new, hipStream_t s, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr);
// Fused CG iteration: one kernel per iteration for chains whose workgroups own whole
// lattice rows (see cg_iter_eligible).  Slot k applies the previous iteration's step
// (r -= alpha s, x += alpha p, with the squared norm of the new residual predicted from the
// previous slot's dot products), forms p = r + beta p, and computes t = D p on the own rows
// and one row beyond, and s = D^dagger t on the own rows, recomputing p two rows beyond the
// own rows from the previous r, s and p (so no other workgroup's output of the same slot is
// read).  Partials of ||t||^2, ||r||^2, Re<r, s>, ||s||^2 go to Q[k & 1].  Mixed precision:
// a reliable update takes two slots (t64 = D x, then r = phi - D^dagger t64).
struct CGIterFields {
    const double2 *phi;
    double2 *x64;
    double2 *t64;     // mixed: FP64 scratch of the residual recomputation
    float4 *x32;      // mixed: FP32 solution increment since the last recomputation
    void *r[2], *s[2], *p[2];  // two buffers each, FP32 float4 (mixed) or FP64 double2 SoA
    const double2 *U64;
    const float *A32;  // FP32 link angles [2][Vtot] (boundary sign folded in as +pi)
    double *Q;        // partial rows [2 slot parities][4][nlog]
    CGState *st;      // [2][nchains]
    double *samples;  // as CGFields::samples
};
// Whether chain ci can use the fused iteration with workgroups of `block` threads, and its
// LDS entries (complex spinors) per workgroup.
bool cg_iter_eligible(const ChainInfo &ci, int block, int *lds_entries);
// Dynamic LDS bytes of the fused iteration for `entries` spinor entries.
size_t cg_iter_lds_bytes(int entries, bool mixed);
void launch_cg_iter(const Geo &g, const CGIterFields &f, bool mixed, int slot, double tol,
                    bool decide_only, int sample, size_t lds_bytes, hipStream_t s,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Lets both instantiations use lds_bytes of dynamic LDS; -1 if the device refuses.
int grant_cg_iter_lds(size_t lds_bytes);

// fin[c][y] = sum of slice y of row's partials of chain c, for the chains above
// kMaxChainBlocks.
void launch_finalize_large(const Geo &g, const double *row, double *fin, hipStream_t s);
// x64 += x32 (end of a mixed solve).
void launch_cg_finish_mixed(const Geo &g, const CGFields &f, hipStream_t s);
// Workgroups of chains not yet converged (st: both state parities) -> out[0..count[0]);
// count[1] = unconverged chains with iterations left (< max_iter).  A chain converged in one
// parity only gets its final state copied into the other.
void launch_compact(const Geo &full, CGState *st, int max_iter, BlockWork *out, int *count,
                    hipStream_t s);
// Persistent solver: one workgroup per chain of chains[0..n), each with at most vmax sites
// (LDS holds p and t: 4 * vmax complex).  Returns -1 if vmax does not fit.
size_t cg_wg_lds_bytes(int vmax, bool mixed);
int launch_cg_wg(const Geo &g, const CGFields &f, bool mixed, const int *chains, int n, int vmax,
                 double tol, double delta, int max_iter, hipStream_t s);
// Grants the persistent solver's dynamic LDS for chains of up to vmax sites ahead of a
// launch (so that no attribute call happens while a stream is captured).  -1 if refused.
int prepare_cg_wg(int vmax, bool mixed);
// Number of converged chains in one state parity -> *out.
void launch_count_converged(const CGState *st_par, int n, int *out, hipStream_t s);

// True residual ||phi - D^dagger D x||^2 per chain into out[c] (t: FP64 spinor scratch).
void launch_true_residual64(const Geo &g, const double2 *U, const double2 *phi, const double2 *x,
                            double2 *t, double *partials, double *out, hipStream_t s);

// ---------------------------------------------------------------- forces
// f = dS_F/dq from chi, xi (Eq. (17)).
void launch_fermion_force(const Geo &g, const double2 *U, const double2 *chi, const double2 *xi,
                          double *f, hipStream_t s);
// F = dS_G/dq (Eq. (16)), plus add[] if add != null (add may alias F).
void launch_gauge_force(const Geo &g, const double *q, const double *add, double *F, hipStream_t s);
// The kick with the gauge force in one kernel: p += c (dS_G/dq + add) (add may be null).
void launch_gauge_kick(const Geo &g, const double *q, const double *add, double c, double *p,
                       hipStream_t s);

// ---------------------------------------------------------------- Hessian-vector products
// W = i v U per link (the links of dD[v], the derivative of D along v).
void launch_weight_links(const Geo &g, const double2 *U, const double *v, double2 *W, hipStream_t s);
// out = S(L1; in1) [+ H(L2; in2)] [- sub]: S the Wilson stencil with links L1 (mass term
// 2 + m0 if mass1, else hopping part only), H the hopping part with links L2 (in2 may be
// null), sub may be null; dagger applies the dagger form to both.
void launch_stencil2(const Geo &g, bool dagger, const double2 *L1, const double2 *in1, bool mass1,
                     const double2 *L2, const double2 *in2, const double2 *sub, double2 *out,
                     hipStream_t s);
// out = scale * (H v): fermion part if chi != null (xi, z1, z2 as in the kernel), gauge part
// if gauge (links q).
void launch_hessian_vector(const Geo &g, const double2 *U, const double *v, const double2 *chi,
                           const double2 *xi, const double2 *z1, const double2 *z2,
                           const double *q, bool gauge, double scale, double *out, hipStream_t s);

// ---------------------------------------------------------------- updates
// out = a + c b over the real link fields, on the sites [site0, site0 + nsites) of g
void launch_axpy_links(const Geo &g, const double *a, double c, const double *b, double *out,
                       hipStream_t s);
void launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------- random numbers
void launch_rng_links(const Geo &g, uint64_t seed, double *q, hipStream_t s);
// momenta (stream 1) and zeta (stream 2) for trajectory traj; per chain
// out[0][c] = 1/2 sum p^2, out[1][c] = zeta^dagger zeta.
void launch_refresh(const Geo &g, uint64_t seed, const uint32_t *traj, double *p, double2 *zeta,
                    bool fermions, double *partials, double *out, hipStream_t s);

// ---------------------------------------------------------------- energies and Metropolis
// Per chain: out[0] = sum 1/2 (p - p0)(p + p0), out[1] = sum (cos theta0 - cos theta),
// out[2] = 1/2 sum p^2, out[3] = sum (1 - cos theta), out[4] = sum (1 - cos theta0),
// out[5] = Re phi^dagger xi (if phi != null), out[6] = sum cos theta.
void launch_energy(const Geo &g, const double *q, const double *q0, const double *p,
                   const double *p0, const double2 *phi, const double2 *xi, double *partials,
                   double *out, hipStream_t s);
// Per chain: out[0] = sum (1 - cos theta), out[1] = sum cos theta,
// out[2] = Re phi^dagger xi (if phi != null).
void launch_gauge_energy(const Geo &g, const double *q, const double2 *phi, const double2 *xi,
                         double *partials, double *out, hipStream_t s);
// One thread per chain: Delta H, Metropolis decision with stream 3.
struct MetroOut {
    double dH, H0, H1, u;
    int accepted, status, pad[2];
};
void launch_metropolis(const Geo &g, uint64_t seed, const uint32_t *traj, const double *esums,
                       const double *rsums, const int *chain_status, MetroOut *out, bool fermions,
                       hipStream_t s);
// Device-side bookkeeping (trajectories that run as one captured graph read their counter
// and write their solver results on the device).
void launch_set_u32(uint32_t *p, uint32_t v, hipStream_t s);
// dst = src, n16 16-byte elements (nontemporal streaming copy)
void launch_stream_copy(const void *src, void *dst, size_t n16, hipStream_t s);
// iterations and stop code (CGState::converged) of every chain's finished solve (state st)
// -> log[2 c + k]
void launch_log_solve(const CGState *st, int nchains, int *log, hipStream_t s);
// status[c] = -3 (iteration cap) or -5 (non-finite residual) from the first of the n logged
// solves (log[k][c][2]) of chain c that stopped unconverged, else 0
void launch_chain_status(const int *log, int n, int nchains, int *status, hipStream_t s);
// p[i] = i for i < n.
void launch_iota(int *p, int n, hipStream_t s);
// q = q0 on the chains whose Metropolis test failed.
void launch_restore(const Geo &g, const MetroOut *m, const double *q0, double *q, hipStream_t s);

}  // namespace shmc
