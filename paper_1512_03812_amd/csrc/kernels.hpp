// Host-side launchers of the HIP kernels (internal interface of the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace shmc {

// Geometry of a batch as the kernels see it.
struct Geo {
    const ChainInfo *chains;  // device, n_chains entries
    const BlockWork *work;    // device, nblocks entries (hardware order)
    int nblocks;              // hardware workgroups of a site kernel
    int nchains;
    int Vtot;
    int block;                // threads per workgroup
};

// Per-chain state of a (possibly mixed-precision) CG solve, device resident.
struct CGState {
    double rho;       // ||r||^2 of the current residual
    double rho_prev;  // ||r||^2 one iteration earlier
    double pAp;       // ||D p||^2 = <p, D^dagger D p>
    double alpha, beta;
    double target;    // tol^2 ||phi||^2
    double phi2;      // ||phi||^2
    double rmax2;     // mixed: ||r||^2 at the last FP64 residual recomputation
    double delta2;    // mixed: reliable-update trigger factor squared
    int iters;        // CG iterations done
    int converged;    // 1 once the stopping test passed
    int update;       // mixed: 1 if the next iteration slot is an FP64 residual recomputation
    int n_updates;    // mixed: FP64 recomputations done
    int pad[6];
};
static_assert(sizeof(CGState) % 16 == 0, "CGState alignment");

// Scratch for per-chain reductions.
struct Reduce {
    double *partials;   // [kMaxReduce][nblocks] logical-ordered block partials
    unsigned *counters; // [nchains] arrival counters (self-resetting)
};
constexpr int kMaxReduce = 8;

// ---------------------------------------------------------------- layout
// to_native: nat <- lex, else lex <- nat
void launch_pack_links(const Geo &g, double *lex, double *nat, bool to_native, hipStream_t s);
void launch_pack_spinor(const Geo &g, double2 *lex, double2 *nat, bool to_native, hipStream_t s);

// ---------------------------------------------------------------- links
// U = exp(i q) with the antiperiodic sign on the t-links leaving the last time slice;
// U32 (may be null) receives the FP32 copy.
void launch_make_links(const Geo &g, const double *q, double2 *U64, float2 *U32, hipStream_t s);

// ---------------------------------------------------------------- Dirac operator
void launch_dslash64(const Geo &g, const double2 *U, const double2 *in, double2 *out, bool dagger,
                     hipStream_t s);

// ---------------------------------------------------------------- CG on D^dagger D
// x = 0, r = phi, ||phi||^2 -> state (rho, target = tol^2 ||phi||^2, converged if phi == 0).
void launch_cg_init64(const Geo &g, const Reduce &red, const double2 *phi, double2 *x, double2 *r,
                      CGState *st, double tol, double delta, hipStream_t s);
// One FP64 iteration: (p_new = r + beta p_old; t = D p_new; ||t||^2 -> alpha) then
// (x += alpha p_new; r -= alpha D^dagger t; ||r||^2 -> beta, convergence).
void launch_cg_step64(const Geo &g, const Reduce &red, const double2 *U, double2 *x, double2 *r,
                      const double2 *p_old, double2 *p_new, double2 *t, CGState *st, hipStream_t s);
// Mixed precision: FP32 iteration with FP64 reliable updates folded into the same slots.
struct MixedFields {
    const double2 *phi;  // FP64 right-hand side
    double2 *x64;        // FP64 accumulated solution
    double2 *t64;        // FP64 scratch (D y in a residual recomputation)
    float2 *x32, *r32, *t32;
};
void launch_cg_init_mixed(const Geo &g, const Reduce &red, const MixedFields &m, CGState *st,
                          double tol, double delta, hipStream_t s);
void launch_cg_step_mixed(const Geo &g, const Reduce &red, const double2 *U64, const float2 *U32,
                          const MixedFields &m, const float2 *p_old, float2 *p_new, CGState *st,
                          hipStream_t s);
// x64 += x32 for chains that stopped between recomputations (none in exact arithmetic);
// also used at the end of a mixed solve.
void launch_cg_finish_mixed(const Geo &g, const MixedFields &m, const CGState *st, hipStream_t s);
// True residual ||phi - D^dagger D x||^2 per chain into out[c] (uses t as scratch).
void launch_true_residual64(const Geo &g, const Reduce &red, const double2 *U, const double2 *phi,
                            const double2 *x, double2 *t, double *out, hipStream_t s);

// ---------------------------------------------------------------- forces
// f = dS_F/dq from chi, xi (Eq. (17)).
void launch_fermion_force(const Geo &g, const double2 *U, const double2 *chi, const double2 *xi,
                          double *f, hipStream_t s);
// F = dS_G/dq (Eq. (16)), plus add[] if add != null.
void launch_gauge_force(const Geo &g, const double *q, const double *add, double *F, hipStream_t s);

// ---------------------------------------------------------------- updates
void launch_axpy_links(const Geo &g, const double *a, double c, const double *b, double *out,
                       hipStream_t s);  // out = a + c b over the real link fields
void launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------- random numbers
void launch_rng_links(const Geo &g, uint64_t seed, double *q, hipStream_t s);
// momenta (stream 1) and zeta (stream 2) for trajectory traj; partial energies
// 1/2 sum p^2 -> sums[0][c], zeta^dagger zeta -> sums[1][c].
void launch_refresh(const Geo &g, const Reduce &red, uint64_t seed, uint32_t traj, double *p,
                    double2 *zeta, bool fermions, double *sums, hipStream_t s);

// ---------------------------------------------------------------- energies and Metropolis
// Per chain: sums[0] = sum 1/2 (p - p0)(p + p0), sums[1] = sum (cos theta0 - cos theta),
// sums[2] = 1/2 sum p^2, sums[3] = sum (1 - cos theta), sums[4] = sum (1 - cos theta0),
// sums[5] = Re phi^dagger xi (if phi != null), sums[6] = sum cos theta.
void launch_energy(const Geo &g, const Reduce &red, const double *q, const double *q0,
                   const double *p, const double *p0, const double2 *phi, const double2 *xi,
                   double *sums, hipStream_t s);
// Per chain: S_G-type sums only: sums[0] = sum (1 - cos theta), sums[1] = sum cos theta,
// sums[2] = Re phi^dagger xi (if phi != null).
void launch_gauge_energy(const Geo &g, const Reduce &red, const double *q, const double2 *phi,
                         const double2 *xi, double *sums, hipStream_t s);
// One thread per chain: Delta H, Metropolis decision with stream 3.
struct MetroOut {
    double dH, H0, H1, u;
    int accepted, status, pad[2];
};
void launch_metropolis(const Geo &g, uint64_t seed, uint32_t traj, const double *esums,
                       const double *rsums, const int *chain_status, MetroOut *out, bool fermions,
                       hipStream_t s);
// q = q0 on the chains whose Metropolis test failed.
void launch_restore(const Geo &g, const MetroOut *m, const double *q0, double *q, hipStream_t s);

}  // namespace shmc
