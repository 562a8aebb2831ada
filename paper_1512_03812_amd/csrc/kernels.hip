// HIP kernels (gfx950) of the Schwinger-model HMC hot path.
//
// Every site kernel runs one thread per lattice site.  Workgroup b handles the sites
// [work[b].start, work[b].start + blockDim) of chain work[b].chain; the host permutes
// the table so that each XCD receives a contiguous range of sites (its L2 then holds
// the neighbouring rows of the stencil).  Per-chain sums use a deterministic two-level
// tree: a wavefront shuffle + LDS reduction per workgroup, then the last workgroup of
// the chain to arrive (agent-scope atomic counter) adds the chain's block partials in
// a fixed order.  No floating-point atomics are used, so every result is bitwise
// reproducible run to run.
#include <math.h>

#include "kernels.hpp"

namespace shmc {

constexpr int kMaxWaves = 1024 / 64;

// ================================================================ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sums NV values over the workgroup; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (&sh)[NV][kMaxWaves]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = 0.0;
            for (int w = 0; w < nw; ++w) a += sh[k][w];
            v[k] = a;
        }
    }
    __syncthreads();
}

// Per-chain reduction.  Returns true in the last-arriving workgroup of the chain, whose
// thread 0 then holds the chain totals in tot[].  All workgroups of a chain must call it.
template <int NV>
__device__ bool chain_reduce(double (&v)[NV], const ChainInfo &ci, const BlockWork &w,
                             const Reduce &red, int nlog, double (&tot)[NV]) {
    __shared__ double sh[NV][kMaxWaves];
    __shared__ int is_last;
    block_sum<NV>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            __hip_atomic_store(&red.partials[(size_t)k * nlog + w.logical], v[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        unsigned prev = __hip_atomic_fetch_add(&red.counters[w.chain], 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        is_last = (prev == (unsigned)(ci.nblocks - 1)) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return false;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        acc[k] = 0.0;
        for (int j = threadIdx.x; j < ci.nblocks; j += blockDim.x)
            acc[k] += __hip_atomic_load(&red.partials[(size_t)k * nlog + ci.block0 + j],
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum<NV>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] = acc[k];
        __hip_atomic_store(&red.counters[w.chain], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

// ================================================================ stencil
struct Nbr {
    int xp, xm, tp, tm;  // flat indices of n+x, n-x, n+t, n-t
};

__device__ __forceinline__ Nbr neighbours(const ChainInfo &ci, const Site &s) {
    Nbr n;
    n.xp = flat_of(ci, wrap_inc(s.x, ci.Lx), s.t);
    n.xm = flat_of(ci, wrap_dec(s.x, ci.Lx), s.t);
    n.tp = flat_of(ci, s.x, wrap_inc(s.t, ci.Lt));
    n.tm = flat_of(ci, s.x, wrap_dec(s.t, ci.Lt));
    return n;
}

// (D a)(n) or (D^dagger a)(n) at one site, Sec. 3.  own0/own1: a(n); load(f, b0, b1)
// fetches a at flat index f.  The hopping projectors (1 -/+ sigma_mu) have rank one:
//   (1 + s sigma_1) v = (w, s w)     with w = v0 + s v1
//   (1 + s sigma_2) v = (w, s i w)   with w = v0 - s i v1
// D uses s = -1 on the forward hop and s = +1 on the backward hop; D^dagger the reverse.
template <typename T, bool DAG, typename Load>
__device__ __forceinline__ void dslash_site(const Nbr &nb, int flat, int Vtot,
                                            const cplx_t<T> *__restrict__ U, cplx_t<T> own0,
                                            cplx_t<T> own1, T mass, Load load, cplx_t<T> &o0,
                                            cplx_t<T> &o1) {
    using C = cplx_t<T>;
    constexpr T sf = DAG ? T(1) : T(-1);  // sign on the forward hop; backward is -sf
    const C uxf = U[flat], utf = U[Vtot + flat], uxb = U[nb.xm], utb = U[Vtot + nb.tm];
    C b0, b1;
    load(nb.xp, b0, b1);
    const C wxf = cmul(uxf, cadd(b0, cscale(b1, sf)));
    load(nb.xm, b0, b1);
    const C wxb = cmulc(uxb, csub(b0, cscale(b1, sf)));
    load(nb.tp, b0, b1);
    const C wtf = cmul(utf, csub(b0, cscale(cmuli(b1), sf)));
    load(nb.tm, b0, b1);
    const C wtb = cmulc(utb, cadd(b0, cscale(cmuli(b1), sf)));
    const C sum0 = cadd(cadd(wxf, wxb), cadd(wtf, wtb));
    const C sum1 = cscale(cadd(csub(wxf, wxb), cmuli(csub(wtf, wtb))), sf);
    o0 = csub(cscale(own0, mass), cscale(sum0, T(0.5)));
    o1 = csub(cscale(own1, mass), cscale(sum1, T(0.5)));
}

__device__ __forceinline__ double norm2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double norm2(float2 a) {
    return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}

#define SITE_PROLOGUE                                  \
    const BlockWork w = g.work[blockIdx.x];            \
    const ChainInfo ci = g.chains[w.chain];            \
    const int local = w.start + (int)threadIdx.x;      \
    const bool valid = local < ci.V;                   \
    const int Vtot = g.Vtot;                           \
    (void)Vtot;

// ================================================================ layout
__global__ void k_pack_links(Geo g, double *__restrict__ lex, double *__restrict__ nat,
                             int to_native) {
    SITE_PROLOGUE
    if (!valid) return;
    const Site s = decode_site(ci, local);
    const size_t l = 2 * ((size_t)ci.off + s.x + (size_t)ci.Lx * s.t);
    for (int mu = 0; mu < 2; ++mu) {
        if (to_native) nat[(size_t)mu * Vtot + s.flat] = lex[l + mu];
        else lex[l + mu] = nat[(size_t)mu * Vtot + s.flat];
    }
}

__global__ void k_pack_spinor(Geo g, double2 *__restrict__ lex, double2 *__restrict__ nat,
                              int to_native) {
    SITE_PROLOGUE
    if (!valid) return;
    const Site s = decode_site(ci, local);
    const size_t l = 2 * ((size_t)ci.off + s.x + (size_t)ci.Lx * s.t);
    for (int sp = 0; sp < 2; ++sp) {
        if (to_native) nat[(size_t)sp * Vtot + s.flat] = lex[l + sp];
        else lex[l + sp] = nat[(size_t)sp * Vtot + s.flat];
    }
}

void launch_pack_links(const Geo &g, double *lex, double *nat, bool to_native, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_links, dim3(g.nblocks), dim3(g.block), 0, s, g,
                       lex, nat, to_native ? 1 : 0);
}
void launch_pack_spinor(const Geo &g, double2 *lex, double2 *nat, bool to_native,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_pack_spinor, dim3(g.nblocks), dim3(g.block), 0, s, g, lex, nat,
                       to_native ? 1 : 0);
}

// ================================================================ links
// U_mu(n) = exp(i q_mu(n)); the t-link leaving the last time slice carries the
// antiperiodic fermion boundary sign.
__global__ void k_make_links(Geo g, const double *__restrict__ q, double2 *__restrict__ U64,
                             float2 *__restrict__ U32) {
    SITE_PROLOGUE
    if (!valid) return;
    const Site s = decode_site(ci, local);
    for (int mu = 0; mu < 2; ++mu) {
        double sn, cs;
        sincos(q[(size_t)mu * Vtot + s.flat], &sn, &cs);
        if (mu == 1 && s.t == ci.Lt - 1) { sn = -sn; cs = -cs; }
        U64[(size_t)mu * Vtot + s.flat] = make_double2(cs, sn);
        if (U32) U32[(size_t)mu * Vtot + s.flat] = make_float2((float)cs, (float)sn);
    }
}

void launch_make_links(const Geo &g, const double *q, double2 *U64, float2 *U32, hipStream_t s) {
    hipLaunchKernelGGL(k_make_links, dim3(g.nblocks), dim3(g.block), 0, s, g, q, U64, U32);
}

// ================================================================ Dirac operator
template <bool DAG>
__global__ void k_dslash64(Geo g, const double2 *__restrict__ U, const double2 *__restrict__ in,
                           double2 *__restrict__ out) {
    SITE_PROLOGUE
    if (!valid) return;
    const Site s = decode_site(ci, local);
    const Nbr nb = neighbours(ci, s);
    auto load = [&](int f, double2 &b0, double2 &b1) { b0 = in[f]; b1 = in[(size_t)Vtot + f]; };
    double2 o0, o1;
    dslash_site<double, DAG>(nb, s.flat, Vtot, U, in[s.flat], in[(size_t)Vtot + s.flat],
                             2.0 + ci.m0, load, o0, o1);
    out[s.flat] = o0;
    out[(size_t)Vtot + s.flat] = o1;
}

void launch_dslash64(const Geo &g, const double2 *U, const double2 *in, double2 *out, bool dagger,
                     hipStream_t s) {
    if (dagger) hipLaunchKernelGGL(k_dslash64<true>, dim3(g.nblocks), dim3(g.block), 0, s, g, U, in, out);
    else hipLaunchKernelGGL(k_dslash64<false>, dim3(g.nblocks), dim3(g.block), 0, s, g, U, in, out);
}

// ================================================================ CG, FP64
__global__ void k_cg_init64(Geo g, Reduce red, const double2 *__restrict__ phi,
                            double2 *__restrict__ x, double2 *__restrict__ r, CGState *st,
                            double tol, double delta) {
    SITE_PROLOGUE
    double v[1] = {0.0};
    if (valid) {
        const int f = ci.off + local;
        for (int sp = 0; sp < 2; ++sp) {
            const double2 a = phi[(size_t)sp * Vtot + f];
            r[(size_t)sp * Vtot + f] = a;
            x[(size_t)sp * Vtot + f] = make_double2(0.0, 0.0);
            v[0] += norm2(a);
        }
    }
    double tot[1];
    if (chain_reduce<1>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        CGState &S = st[w.chain];
        S.phi2 = tot[0];
        S.rho = tot[0];
        S.rho_prev = tot[0];
        S.rmax2 = tot[0];
        S.target = tol * tol * tot[0];
        S.delta2 = delta * delta;
        S.alpha = 0.0;
        S.beta = 0.0;
        S.pAp = 0.0;
        S.iters = 0;
        S.update = 0;
        S.n_updates = 0;
        S.converged = (tot[0] <= S.target) ? 1 : 0;
    }
}

// p_new = r + beta p_old (p_new = r on the first iteration), t = D p_new, ||t||^2 -> alpha.
__global__ void k_cg_step1_64(Geo g, Reduce red, const double2 *__restrict__ U,
                              const double2 *__restrict__ r, const double2 *__restrict__ p_old,
                              double2 *__restrict__ p_new, double2 *__restrict__ t, CGState *st) {
    SITE_PROLOGUE
    const CGState S = st[w.chain];
    if (S.converged) return;
    const bool first = S.iters == 0;
    const double beta = S.beta;
    double v[1] = {0.0};
    if (valid) {
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int f, double2 &b0, double2 &b1) {
            b0 = r[f];
            b1 = r[(size_t)Vtot + f];
            if (!first) {
                const double2 q0 = p_old[f], q1 = p_old[(size_t)Vtot + f];
                b0 = make_double2(b0.x + beta * q0.x, b0.y + beta * q0.y);
                b1 = make_double2(b1.x + beta * q1.x, b1.y + beta * q1.y);
            }
        };
        double2 a0, a1, o0, o1;
        load(s.flat, a0, a1);
        dslash_site<double, false>(nb, s.flat, Vtot, U, a0, a1, 2.0 + ci.m0, load, o0, o1);
        p_new[s.flat] = a0;
        p_new[(size_t)Vtot + s.flat] = a1;
        t[s.flat] = o0;
        t[(size_t)Vtot + s.flat] = o1;
        v[0] = norm2(o0) + norm2(o1);
    }
    double tot[1];
    if (chain_reduce<1>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        st[w.chain].pAp = tot[0];
        st[w.chain].alpha = S.rho / tot[0];
    }
}

// x += alpha p; r -= alpha D^dagger t; ||r||^2 -> rho, beta, convergence.
__global__ void k_cg_step2_64(Geo g, Reduce red, const double2 *__restrict__ U,
                              double2 *__restrict__ x, double2 *__restrict__ r,
                              const double2 *__restrict__ p, const double2 *__restrict__ t,
                              CGState *st) {
    SITE_PROLOGUE
    const CGState S = st[w.chain];
    if (S.converged) return;
    const double alpha = S.alpha;
    double v[1] = {0.0};
    if (valid) {
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int f, double2 &b0, double2 &b1) { b0 = t[f]; b1 = t[(size_t)Vtot + f]; };
        double2 a0, a1;
        dslash_site<double, true>(nb, s.flat, Vtot, U, t[s.flat], t[(size_t)Vtot + s.flat],
                                  2.0 + ci.m0, load, a0, a1);
        const double2 Ap[2] = {a0, a1};
        for (int sp = 0; sp < 2; ++sp) {
            const size_t f = (size_t)sp * Vtot + s.flat;
            const double2 pp = p[f];
            double2 xx = x[f], rr = r[f];
            xx.x += alpha * pp.x; xx.y += alpha * pp.y;
            rr.x -= alpha * Ap[sp].x; rr.y -= alpha * Ap[sp].y;
            x[f] = xx;
            r[f] = rr;
            v[0] += norm2(rr);
        }
    }
    double tot[1];
    if (chain_reduce<1>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        CGState &T = st[w.chain];
        T.iters = S.iters + 1;
        T.rho_prev = S.rho;
        T.rho = tot[0];
        if (tot[0] <= S.target) T.converged = 1;
        else T.beta = tot[0] / S.rho;
    }
}

void launch_cg_init64(const Geo &g, const Reduce &red, const double2 *phi, double2 *x, double2 *r,
                      CGState *st, double tol, double delta, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init64, dim3(g.nblocks), dim3(g.block), 0, s, g, red, phi, x, r, st,
                       tol, delta);
}

void launch_cg_step64(const Geo &g, const Reduce &red, const double2 *U, double2 *x, double2 *r,
                      const double2 *p_old, double2 *p_new, double2 *t, CGState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_step1_64, dim3(g.nblocks), dim3(g.block), 0, s, g, red, U, r, p_old,
                       p_new, t, st);
    hipLaunchKernelGGL(k_cg_step2_64, dim3(g.nblocks), dim3(g.block), 0, s, g, red, U, x, r, p_new,
                       t, st);
}

// ================================================================ CG, mixed precision
// FP32 iterations; when the FP32 residual has dropped by delta since the last FP64
// recomputation (or reached the target), the next iteration slot recomputes
// r = phi - D^dagger D (x64 + x32) in FP64, folds x32 into x64 and restarts the FP32
// residual from it (reliable update).  Convergence is only declared on that FP64 residual.
__global__ void k_cg_init_mixed(Geo g, Reduce red, MixedFields m, CGState *st, double tol,
                                double delta) {
    SITE_PROLOGUE
    double v[1] = {0.0};
    if (valid) {
        const int f = ci.off + local;
        for (int sp = 0; sp < 2; ++sp) {
            const size_t k = (size_t)sp * Vtot + f;
            const double2 a = m.phi[k];
            m.x64[k] = make_double2(0.0, 0.0);
            m.x32[k] = make_float2(0.f, 0.f);
            m.r32[k] = make_float2((float)a.x, (float)a.y);
            v[0] += norm2(a);
        }
    }
    double tot[1];
    if (chain_reduce<1>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        CGState &S = st[w.chain];
        S.phi2 = tot[0];
        S.rho = tot[0];
        S.rho_prev = tot[0];
        S.rmax2 = tot[0];
        S.target = tol * tol * tot[0];
        S.delta2 = delta * delta;
        S.alpha = 0.0;
        S.beta = 0.0;
        S.pAp = 0.0;
        S.iters = 0;
        S.update = 0;
        S.n_updates = 0;
        S.converged = (tot[0] <= S.target) ? 1 : 0;
    }
}

__global__ void k_cg_step1_mixed(Geo g, Reduce red, const double2 *__restrict__ U64,
                                 const float2 *__restrict__ U32, MixedFields m,
                                 const float2 *__restrict__ p_old, float2 *__restrict__ p_new,
                                 CGState *st) {
    SITE_PROLOGUE
    const CGState S = st[w.chain];
    if (S.converged) return;
    if (S.update) {
        // FP64 residual recomputation, first half: t64 = D (x64 + x32); p carried over.
        if (!valid) return;
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int f, double2 &b0, double2 &b1) {
            const double2 y0 = m.x64[f], y1 = m.x64[(size_t)Vtot + f];
            const float2 z0 = m.x32[f], z1 = m.x32[(size_t)Vtot + f];
            b0 = make_double2(y0.x + (double)z0.x, y0.y + (double)z0.y);
            b1 = make_double2(y1.x + (double)z1.x, y1.y + (double)z1.y);
        };
        double2 a0, a1, o0, o1;
        load(s.flat, a0, a1);
        dslash_site<double, false>(nb, s.flat, Vtot, U64, a0, a1, 2.0 + ci.m0, load, o0, o1);
        m.t64[s.flat] = o0;
        m.t64[(size_t)Vtot + s.flat] = o1;
        if (S.iters > 0) {
            p_new[s.flat] = p_old[s.flat];
            p_new[(size_t)Vtot + s.flat] = p_old[(size_t)Vtot + s.flat];
        }
        return;
    }
    const bool first = S.iters == 0;
    const float beta = (float)S.beta;
    double v[1] = {0.0};
    if (valid) {
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int f, float2 &b0, float2 &b1) {
            b0 = m.r32[f];
            b1 = m.r32[(size_t)Vtot + f];
            if (!first) {
                const float2 q0 = p_old[f], q1 = p_old[(size_t)Vtot + f];
                b0 = make_float2(b0.x + beta * q0.x, b0.y + beta * q0.y);
                b1 = make_float2(b1.x + beta * q1.x, b1.y + beta * q1.y);
            }
        };
        float2 a0, a1, o0, o1;
        load(s.flat, a0, a1);
        dslash_site<float, false>(nb, s.flat, Vtot, U32, a0, a1, 2.0f + (float)ci.m0, load, o0, o1);
        p_new[s.flat] = a0;
        p_new[(size_t)Vtot + s.flat] = a1;
        m.t32[s.flat] = o0;
        m.t32[(size_t)Vtot + s.flat] = o1;
        v[0] = norm2(o0) + norm2(o1);
    }
    double tot[1];
    if (chain_reduce<1>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        st[w.chain].pAp = tot[0];
        st[w.chain].alpha = S.rho / tot[0];
    }
}

__global__ void k_cg_step2_mixed(Geo g, Reduce red, const double2 *__restrict__ U64,
                                 const float2 *__restrict__ U32, MixedFields m,
                                 const float2 *__restrict__ p, CGState *st) {
    SITE_PROLOGUE
    const CGState S = st[w.chain];
    if (S.converged) return;
    double v[1] = {0.0};
    double tot[1];
    if (S.update) {
        // second half: r64 = phi - D^dagger t64; x64 += x32; x32 = 0; r32 = r64.
        if (valid) {
            const Site s = decode_site(ci, local);
            const Nbr nb = neighbours(ci, s);
            auto load = [&](int f, double2 &b0, double2 &b1) {
                b0 = m.t64[f];
                b1 = m.t64[(size_t)Vtot + f];
            };
            double2 a0, a1;
            dslash_site<double, true>(nb, s.flat, Vtot, U64, m.t64[s.flat],
                                      m.t64[(size_t)Vtot + s.flat], 2.0 + ci.m0, load, a0, a1);
            const double2 Ay[2] = {a0, a1};
            for (int sp = 0; sp < 2; ++sp) {
                const size_t f = (size_t)sp * Vtot + s.flat;
                const double2 ph = m.phi[f];
                const double2 rr = make_double2(ph.x - Ay[sp].x, ph.y - Ay[sp].y);
                const double2 xx = m.x64[f];
                const float2 zz = m.x32[f];
                m.x64[f] = make_double2(xx.x + (double)zz.x, xx.y + (double)zz.y);
                m.x32[f] = make_float2(0.f, 0.f);
                m.r32[f] = make_float2((float)rr.x, (float)rr.y);
                v[0] += norm2(rr);
            }
        }
        if (chain_reduce<1>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
            CGState &T = st[w.chain];
            T.update = 0;
            T.n_updates = S.n_updates + 1;
            T.rmax2 = tot[0];
            T.rho = tot[0];
            if (tot[0] <= S.target) T.converged = 1;
            else T.beta = tot[0] / S.rho_prev;
        }
        return;
    }
    const float alpha = (float)S.alpha;
    if (valid) {
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int f, float2 &b0, float2 &b1) {
            b0 = m.t32[f];
            b1 = m.t32[(size_t)Vtot + f];
        };
        float2 a0, a1;
        dslash_site<float, true>(nb, s.flat, Vtot, U32, m.t32[s.flat], m.t32[(size_t)Vtot + s.flat],
                                 2.0f + (float)ci.m0, load, a0, a1);
        const float2 Ap[2] = {a0, a1};
        for (int sp = 0; sp < 2; ++sp) {
            const size_t f = (size_t)sp * Vtot + s.flat;
            const float2 pp = p[f];
            float2 xx = m.x32[f], rr = m.r32[f];
            xx.x += alpha * pp.x; xx.y += alpha * pp.y;
            rr.x -= alpha * Ap[sp].x; rr.y -= alpha * Ap[sp].y;
            m.x32[f] = xx;
            m.r32[f] = rr;
            v[0] += norm2(rr);
        }
    }
    if (chain_reduce<1>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        CGState &T = st[w.chain];
        T.iters = S.iters + 1;
        T.rho_prev = S.rho;
        T.rho = tot[0];
        T.beta = tot[0] / S.rho;
        if (tot[0] <= S.target || tot[0] <= S.delta2 * S.rmax2) T.update = 1;
    }
}

__global__ void k_cg_finish_mixed(Geo g, MixedFields m, const CGState *st) {
    SITE_PROLOGUE
    if (!valid) return;
    const int f = ci.off + local;
    for (int sp = 0; sp < 2; ++sp) {
        const size_t k = (size_t)sp * Vtot + f;
        const double2 xx = m.x64[k];
        const float2 zz = m.x32[k];
        m.x64[k] = make_double2(xx.x + (double)zz.x, xx.y + (double)zz.y);
        m.x32[k] = make_float2(0.f, 0.f);
    }
}

void launch_cg_init_mixed(const Geo &g, const Reduce &red, const MixedFields &m, CGState *st,
                          double tol, double delta, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init_mixed, dim3(g.nblocks), dim3(g.block), 0, s, g, red, m, st, tol,
                       delta);
}

void launch_cg_step_mixed(const Geo &g, const Reduce &red, const double2 *U64, const float2 *U32,
                          const MixedFields &m, const float2 *p_old, float2 *p_new, CGState *st,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_cg_step1_mixed, dim3(g.nblocks), dim3(g.block), 0, s, g, red, U64, U32, m,
                       p_old, p_new, st);
    hipLaunchKernelGGL(k_cg_step2_mixed, dim3(g.nblocks), dim3(g.block), 0, s, g, red, U64, U32, m,
                       p_new, st);
}

void launch_cg_finish_mixed(const Geo &g, const MixedFields &m, const CGState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_finish_mixed, dim3(g.nblocks), dim3(g.block), 0, s, g, m, st);
}

// ||phi - D^dagger t||^2 per chain, t = D x computed before.
__global__ void k_residual64(Geo g, Reduce red, const double2 *__restrict__ U,
                             const double2 *__restrict__ phi, const double2 *__restrict__ t,
                             double *out) {
    SITE_PROLOGUE
    double v[1] = {0.0};
    if (valid) {
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int f, double2 &b0, double2 &b1) { b0 = t[f]; b1 = t[(size_t)Vtot + f]; };
        double2 a0, a1;
        dslash_site<double, true>(nb, s.flat, Vtot, U, t[s.flat], t[(size_t)Vtot + s.flat],
                                  2.0 + ci.m0, load, a0, a1);
        const double2 ph0 = phi[s.flat], ph1 = phi[(size_t)Vtot + s.flat];
        v[0] = norm2(make_double2(ph0.x - a0.x, ph0.y - a0.y)) +
               norm2(make_double2(ph1.x - a1.x, ph1.y - a1.y));
    }
    double tot[1];
    if (chain_reduce<1>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) out[w.chain] = tot[0];
}

void launch_true_residual64(const Geo &g, const Reduce &red, const double2 *U, const double2 *phi,
                            const double2 *x, double2 *t, double *out, hipStream_t s) {
    launch_dslash64(g, U, x, t, false, s);
    hipLaunchKernelGGL(k_residual64, dim3(g.nblocks), dim3(g.block), 0, s, g, red, U, phi, t, out);
}

// ================================================================ forces
// f(n, mu) = -Im[chi^dagger(n) (1 - sigma_mu) U_mu(n) xi(n+mu)
//                - chi^dagger(n+mu) (1 + sigma_mu) U_mu^dagger(n) xi(n)]      (Eq. (17))
// With the rank-one projectors:
//   mu = x: chi^dagger (1 - sigma_1) v = conj(chi0 - chi1) (v0 - v1),
//           chi^dagger (1 + sigma_1) v = conj(chi0 + chi1) (v0 + v1)
//   mu = t: chi^dagger (1 - sigma_2) v = conj(chi0 + i chi1) (v0 + i v1),
//           chi^dagger (1 + sigma_2) v = conj(chi0 - i chi1) (v0 - i v1)
__global__ void k_fermion_force(Geo g, const double2 *__restrict__ U,
                                const double2 *__restrict__ chi, const double2 *__restrict__ xi,
                                double *__restrict__ f) {
    SITE_PROLOGUE
    if (!valid) return;
    const Site s = decode_site(ci, local);
    const int nxp = flat_of(ci, wrap_inc(s.x, ci.Lx), s.t);
    const int ntp = flat_of(ci, s.x, wrap_inc(s.t, ci.Lt));
    const double2 c0 = chi[s.flat], c1 = chi[(size_t)Vtot + s.flat];
    const double2 x0 = xi[s.flat], x1 = xi[(size_t)Vtot + s.flat];
    {   // mu = x
        const double2 u = U[s.flat];
        const double2 cn0 = chi[nxp], cn1 = chi[(size_t)Vtot + nxp];
        const double2 xn0 = xi[nxp], xn1 = xi[(size_t)Vtot + nxp];
        const double2 term1 = cmulc(csub(c0, c1), cmul(u, csub(xn0, xn1)));
        const double2 term2 = cmulc(cadd(cn0, cn1), cmulc(u, cadd(x0, x1)));
        f[s.flat] = term2.y - term1.y;
    }
    {   // mu = t
        const double2 u = U[(size_t)Vtot + s.flat];
        const double2 cn0 = chi[ntp], cn1 = chi[(size_t)Vtot + ntp];
        const double2 xn0 = xi[ntp], xn1 = xi[(size_t)Vtot + ntp];
        const double2 term1 = cmulc(cadd(c0, cmuli(c1)), cmul(u, cadd(xn0, cmuli(xn1))));
        const double2 term2 = cmulc(csub(cn0, cmuli(cn1)), cmulc(u, csub(x0, cmuli(x1))));
        f[(size_t)Vtot + s.flat] = term2.y - term1.y;
    }
}

void launch_fermion_force(const Geo &g, const double2 *U, const double2 *chi, const double2 *xi,
                          double *f, hipStream_t s) {
    hipLaunchKernelGGL(k_fermion_force, dim3(g.nblocks), dim3(g.block), 0, s, g, U, chi, xi, f);
}

// plaquette angle theta(x, t) = q_x(n) + q_t(n + x) - q_x(n + t) - q_t(n)
__device__ __forceinline__ double plaq_angle(const ChainInfo &ci, const double *__restrict__ q,
                                             int Vtot, int x, int t) {
    const int n = flat_of(ci, x, t);
    const int nx = flat_of(ci, wrap_inc(x, ci.Lx), t);
    const int nt = flat_of(ci, x, wrap_inc(t, ci.Lt));
    return q[n] + q[(size_t)Vtot + nx] - q[nt] - q[(size_t)Vtot + n];
}

// dS_G/dq: F_x(n) = beta [sin theta(n) - sin theta(n - t)], F_t(n) = beta [sin theta(n - x)
// - sin theta(n)] -- Eq. (16) with P read as P_{mu nu}(n), whose angle is -theta for mu = t.
__global__ void k_gauge_force(Geo g, const double *__restrict__ q, const double *__restrict__ add,
                              double *__restrict__ F) {
    SITE_PROLOGUE
    if (!valid) return;
    const Site s = decode_site(ci, local);
    const double th = plaq_angle(ci, q, Vtot, s.x, s.t);
    const double th_mt = plaq_angle(ci, q, Vtot, s.x, wrap_dec(s.t, ci.Lt));
    const double th_mx = plaq_angle(ci, q, Vtot, wrap_dec(s.x, ci.Lx), s.t);
    const double sn = sin(th);
    double fx = ci.beta * (sn - sin(th_mt));
    double ft = ci.beta * (sin(th_mx) - sn);
    if (add) {
        fx += add[s.flat];
        ft += add[(size_t)Vtot + s.flat];
    }
    F[s.flat] = fx;
    F[(size_t)Vtot + s.flat] = ft;
}

void launch_gauge_force(const Geo &g, const double *q, const double *add, double *F, hipStream_t s) {
    hipLaunchKernelGGL(k_gauge_force, dim3(g.nblocks), dim3(g.block), 0, s, g, q, add, F);
}

// ================================================================ updates
__global__ void k_axpy(const double *__restrict__ a, double c, const double *__restrict__ b,
                       double *__restrict__ out, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = a[i] + c * b[i];
}

void launch_axpy_links(const Geo &g, const double *a, double c, const double *b, double *out,
                       hipStream_t s) {
    const size_t n = 2 * (size_t)g.Vtot;
    const int block = 256;
    size_t grid = (n + block - 1) / block;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)grid), dim3(block), 0, s, a, c, b, out, n);
}

void launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    (void)hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

// ================================================================ random numbers
// Box-Muller pair from Philox words: r = sqrt(-2 log(1 - ua)), (r cos 2 pi ub, r sin 2 pi ub).
__device__ __forceinline__ void gaussian_pair(const U32x4 &w, double &g0, double &g1) {
#pragma clang fp contract(off)
    const double ua = u01_from(w.v[0], w.v[1]), ub = u01_from(w.v[2], w.v[3]);
    const double r = sqrt(-2.0 * log(1.0 - ua));
    const double a = 6.283185307179586 * ub;
    g0 = r * cos(a);
    g1 = r * sin(a);
}

__global__ void k_rng_links(Geo g, uint32_t k0, uint32_t k1, double *__restrict__ q) {
#pragma clang fp contract(off)
    SITE_PROLOGUE
    if (!valid) return;
    const Site s = decode_site(ci, local);
    const uint32_t n = (uint32_t)(s.x + ci.Lx * s.t);
    for (int mu = 0; mu < 2; ++mu) {
        const U32x4 r = philox4x32_10(2 * n + mu, kStreamLinks, 0u, ci.chain_id, k0, k1);
        const double u = u01_from(r.v[0], r.v[1]);
        q[(size_t)mu * Vtot + s.flat] = 3.141592653589793 * (2.0 * u - 1.0);
    }
}

void launch_rng_links(const Geo &g, uint64_t seed, double *q, hipStream_t s) {
    hipLaunchKernelGGL(k_rng_links, dim3(g.nblocks), dim3(g.block), 0, s, g, (uint32_t)seed,
                       (uint32_t)(seed >> 32), q);
}

__global__ void k_refresh(Geo g, Reduce red, uint32_t k0, uint32_t k1, uint32_t traj,
                          double *__restrict__ p, double2 *__restrict__ zeta, int fermions,
                          double *sums) {
#pragma clang fp contract(off)
    SITE_PROLOGUE
    double v[2] = {0.0, 0.0};
    if (valid) {
        const Site s = decode_site(ci, local);
        const uint32_t n = (uint32_t)(s.x + ci.Lx * s.t);
        for (int mu = 0; mu < 2; ++mu) {
            double g0, g1;
            gaussian_pair(philox4x32_10(2 * n + mu, kStreamMomenta, traj, ci.chain_id, k0, k1), g0, g1);
            p[(size_t)mu * Vtot + s.flat] = g0;
            v[0] += 0.5 * g0 * g0;
        }
        if (fermions) {
            for (int sp = 0; sp < 2; ++sp) {
                double g0, g1;
                gaussian_pair(philox4x32_10(2 * n + sp, kStreamPseudofermion, traj, ci.chain_id, k0, k1),
                              g0, g1);
                const double2 z = make_double2(g0 * 0.70710678118654752440, g1 * 0.70710678118654752440);
                zeta[(size_t)sp * Vtot + s.flat] = z;
                v[1] += z.x * z.x + z.y * z.y;
            }
        }
    }
    double tot[2];
    if (chain_reduce<2>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        sums[w.chain] = tot[0];
        sums[g.nchains + w.chain] = tot[1];
    }
}

void launch_refresh(const Geo &g, const Reduce &red, uint64_t seed, uint32_t traj, double *p,
                    double2 *zeta, bool fermions, double *sums, hipStream_t s) {
    hipLaunchKernelGGL(k_refresh, dim3(g.nblocks), dim3(g.block), 0, s, g, red, (uint32_t)seed,
                       (uint32_t)(seed >> 32), traj, p, zeta, fermions ? 1 : 0, sums);
}

// ================================================================ energies
__global__ void k_energy(Geo g, Reduce red, const double *__restrict__ q,
                         const double *__restrict__ q0, const double *__restrict__ p,
                         const double *__restrict__ p0, const double2 *__restrict__ phi,
                         const double2 *__restrict__ xi, double *sums) {
    SITE_PROLOGUE
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (valid) {
        const Site s = decode_site(ci, local);
        for (int mu = 0; mu < 2; ++mu) {
            const double a = p[(size_t)mu * Vtot + s.flat], b = p0[(size_t)mu * Vtot + s.flat];
            v[0] += 0.5 * (a - b) * (a + b);
            v[2] += 0.5 * a * a;
        }
        const double c1 = cos(plaq_angle(ci, q, Vtot, s.x, s.t));
        const double c0 = cos(plaq_angle(ci, q0, Vtot, s.x, s.t));
        v[1] = c0 - c1;
        v[3] = 1.0 - c1;
        v[4] = 1.0 - c0;
        v[6] = c1;
        if (phi) {
            for (int sp = 0; sp < 2; ++sp) {
                const double2 a = phi[(size_t)sp * Vtot + s.flat], b = xi[(size_t)sp * Vtot + s.flat];
                v[5] += a.x * b.x + a.y * b.y;
            }
        }
    }
    double tot[7];
    if (chain_reduce<7>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        for (int k = 0; k < 7; ++k) sums[k * g.nchains + w.chain] = tot[k];
    }
}

void launch_energy(const Geo &g, const Reduce &red, const double *q, const double *q0,
                   const double *p, const double *p0, const double2 *phi, const double2 *xi,
                   double *sums, hipStream_t s) {
    hipLaunchKernelGGL(k_energy, dim3(g.nblocks), dim3(g.block), 0, s, g, red, q, q0, p, p0, phi,
                       xi, sums);
}

__global__ void k_gauge_energy(Geo g, Reduce red, const double *__restrict__ q,
                               const double2 *__restrict__ phi, const double2 *__restrict__ xi,
                               double *sums) {
    SITE_PROLOGUE
    double v[3] = {0, 0, 0};
    if (valid) {
        const Site s = decode_site(ci, local);
        const double c1 = cos(plaq_angle(ci, q, Vtot, s.x, s.t));
        v[0] = 1.0 - c1;
        v[1] = c1;
        if (phi) {
            for (int sp = 0; sp < 2; ++sp) {
                const double2 a = phi[(size_t)sp * Vtot + s.flat], b = xi[(size_t)sp * Vtot + s.flat];
                v[2] += a.x * b.x + a.y * b.y;
            }
        }
    }
    double tot[3];
    if (chain_reduce<3>(v, ci, w, red, g.nblocks, tot) && threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) sums[k * g.nchains + w.chain] = tot[k];
    }
}

void launch_gauge_energy(const Geo &g, const Reduce &red, const double *q, const double2 *phi,
                         const double2 *xi, double *sums, hipStream_t s) {
    hipLaunchKernelGGL(k_gauge_energy, dim3(g.nblocks), dim3(g.block), 0, s, g, red, q, phi, xi,
                       sums);
}

// Delta H = sum 1/2 (p'^2 - p^2) + beta sum (cos theta - cos theta') + (S_F' - S_F), then
// accept iff Delta H <= 0 or u < exp(-Delta H) (Sec. 2.1).
__global__ void k_metropolis(Geo g, uint32_t k0, uint32_t k1, uint32_t traj,
                             const double *__restrict__ es, const double *__restrict__ rs,
                             const int *__restrict__ cstat, MetroOut *out, int fermions) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nchains) return;
    const ChainInfo ci = g.chains[c];
    const int C = g.nchains;
    const double sf1 = fermions ? es[5 * C + c] : 0.0, sf0 = fermions ? rs[C + c] : 0.0;
    const double dH = es[0 * C + c] + ci.beta * es[1 * C + c] + (sf1 - sf0);
    const double H0 = rs[c] + ci.beta * es[4 * C + c] + sf0;
    const double H1 = es[2 * C + c] + ci.beta * es[3 * C + c] + sf1;
    const U32x4 r = philox4x32_10(0u, kStreamMetropolis, traj, ci.chain_id, k0, k1);
    const double u = u01_from(r.v[0], r.v[1]);
    int status = cstat ? cstat[c] : 0;
    if (status == 0 && !isfinite(dH)) status = -5;
    const int acc = status == 0 && (dH <= 0.0 || u < exp(-dH));
    MetroOut m;
    m.dH = dH; m.H0 = H0; m.H1 = H1; m.u = u; m.accepted = acc; m.status = status;
    m.pad[0] = m.pad[1] = 0;
    out[c] = m;
}

void launch_metropolis(const Geo &g, uint64_t seed, uint32_t traj, const double *esums,
                       const double *rsums, const int *chain_status, MetroOut *out, bool fermions,
                       hipStream_t s) {
    const int block = 64;
    hipLaunchKernelGGL(k_metropolis, dim3((g.nchains + block - 1) / block), dim3(block), 0, s, g,
                       (uint32_t)seed, (uint32_t)(seed >> 32), traj, esums, rsums, chain_status, out,
                       fermions ? 1 : 0);
}

__global__ void k_restore(Geo g, const MetroOut *__restrict__ m, const double *__restrict__ q0,
                          double *__restrict__ q) {
    SITE_PROLOGUE
    if (!valid) return;
    if (m[w.chain].accepted) return;
    const int f = ci.off + local;
    q[f] = q0[f];
    q[(size_t)Vtot + f] = q0[(size_t)Vtot + f];
}

void launch_restore(const Geo &g, const MetroOut *m, const double *q0, double *q, hipStream_t s) {
    hipLaunchKernelGGL(k_restore, dim3(g.nblocks), dim3(g.block), 0, s, g, m, q0, q);
}

}  // namespace shmc
