// HIP kernels (gfx950) of the Schwinger-model HMC hot path.
//
// Site kernels: workgroup b handles the half-site indices [start, start + B/2) of both
// parity planes of chain work[b].chain (the stencil neighbours of one plane are the other
// plane's sites at nearby indices); the host permutes the workgroup table so that each XCD
// receives a contiguous range of sites (its L2 then holds the neighbouring rows).
//
// Reductions use no atomics and no cross-workgroup fences: a producer kernel writes one
// partial per workgroup (DPP wavefront sums + LDS), and every consumer workgroup of a
// chain re-adds that chain's partials in a fixed order, so all of them obtain the same,
// bitwise reproducible total.  The kernel boundary provides the visibility.  Totals that
// the host needs go through a one-workgroup-per-chain finalize kernel.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "kernels.hpp"

#include <hip/hip_ext.h>

namespace shmc {

constexpr int kMaxWaves = kMaxBlock / 64;

// ================================================================ reductions
// v plus the value that the DPP control CTRL routes to this lane from another lane of its
// row (every source in range: quad permutations and row rotations).
template <int CTRL> __device__ __forceinline__ double dpp_add_all(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return v + __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// The same for a control applied in the rows of the mask ROWS only; lanes of the other rows
// add 0.
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_add(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return v + __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Wavefront sum in a fixed order through the DPP lane network, with no LDS traffic (2-3 %
// faster CG step kernels than a shuffle tree, whose every step is an LDS permute): sums over
// quads, then over rows of 16 lanes, then two row broadcasts leave the total in lane 63,
// which every lane receives.
__device__ __forceinline__ double wave_sum(double v) {
    v = dpp_add_all<0xb1>(v);     // quad_perm [1,0,3,2]
    v = dpp_add_all<0x4e>(v);     // quad_perm [2,3,0,1]
    v = dpp_add_all<0x124>(v);    // row_ror:4
    v = dpp_add_all<0x128>(v);    // row_ror:8
    v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sums NV values over the workgroup; every thread receives the totals.
template <int NV> __device__ __forceinline__ void block_sum_all(double (&v)[NV]) {
    __shared__ double sh[NV][kMaxWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k][wave] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = 0.0;
        for (int w = 0; w < nw; ++w) a += sh[k][w];
        v[k] = a;
    }
    __syncthreads();
}

// Workgroup sum of one value with one barrier, every thread receiving the total: the
// wavefront sums meet in LDS buffer `buf` (0 or 1) and each thread adds them in a fixed
// order.  Alternating the buffer between consecutive calls makes a second barrier
// unnecessary: a thread can only rewrite a buffer after the other buffer's barrier, which
// every thread reaches after reading it.
__device__ __forceinline__ double block_sum_bcast(double v, int buf) {
    __shared__ double sh[2][kMaxWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    if (lane == 0) sh[buf][wave] = v;
    __syncthreads();
    double a = 0.0;
    for (int w = 0; w < nw; ++w) a += sh[buf][w];
    return a;
}

// One partial per workgroup into row k of partials (k < NV).  It ends its kernel (every
// caller's last use of LDS), so one barrier suffices: the wavefront sums meet in LDS and
// thread 0 adds them in a fixed order.
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *partials, int nlog,
                                               int logical) {
    __shared__ double wsum[NV][kMaxWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) wsum[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = 0.0;
            for (int w = 0; w < nw; ++w) a += wsum[k][w];
            partials[(size_t)k * nlog + logical] = a;
        }
    }
}

// The chain's total of one partial row, identical in every wavefront of the chain: each
// wavefront re-adds the partials of chains of at most kMaxChainBlocks workgroups itself (lane
// l takes partials l, l + 64, ... in order, then the fixed DPP tree of wave_sum), with no LDS
// and no barrier, so the site loads issued before it stay in flight; larger chains re-add the
// kFinSlices slice sums that k_finalize_large wrote after the producer.
__device__ __forceinline__ double chain_total(const double *__restrict__ row,
                                              const double *__restrict__ fin, const ChainInfo &ci,
                                              int chain) {
    double a = 0.0;
    if (ci.nblocks > kMaxChainBlocks) {
        const int l = (int)(threadIdx.x & 63);
        if (l < kFinSlices) a = fin[(size_t)chain * kFinSlices + l];
        return wave_sum(a);
    }
    for (int j = (int)(threadIdx.x & 63); j < ci.nblocks; j += 64) a += row[ci.block0 + j];
    return wave_sum(a);
}

// Slice sums of the partials of chains above kMaxChainBlocks workgroups: workgroup (c, y)
// adds the partials of slice y of chain c (each thread four consecutive ones per pass into
// independent accumulators), in a fixed order, into fin[c][y].
__global__ void k_finalize_large(Geo g, const double *__restrict__ row, double *fin) {
    const ChainInfo ci = g.chains[blockIdx.x];
    if (ci.nblocks <= kMaxChainBlocks) return;
    const int len = (ci.nblocks + kFinSlices - 1) / kFinSlices;
    const int lo = (int)blockIdx.y * len, hi = min(ci.nblocks, lo + len);
    const double *__restrict__ r = row + ci.block0;
    double acc[4] = {0, 0, 0, 0};
    for (int base = lo + 4 * (int)threadIdx.x; base < hi; base += 4 * (int)blockDim.x) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (base + k < hi) acc[k] += r[base + k];
    }
    double v[1] = {(acc[0] + acc[1]) + (acc[2] + acc[3])};
    block_sum_all<1>(v);
    if (threadIdx.x == 0) fin[(size_t)blockIdx.x * kFinSlices + blockIdx.y] = v[0];
}

void launch_finalize_large(const Geo &g, const double *row, double *fin, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_large, dim3(g.nchains, kFinSlices), dim3(256), 0, s, g, row, fin);
}

template <int NV> __global__ void k_finalize(Geo g, const double *__restrict__ partials, double *out) {
    const ChainInfo ci = g.chains[blockIdx.x];
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        v[k] = 0.0;
        for (int j = threadIdx.x; j < ci.nblocks; j += blockDim.x)
            v[k] += partials[(size_t)k * g.nlog + ci.block0 + j];
    }
    block_sum_all<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) out[(size_t)k * g.nchains + blockIdx.x] = v[k];
    }
}

template <int NV> void launch_finalize(const Geo &g, const double *partials, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize<NV>, dim3(g.nchains), dim3(256), 0, s, g, partials, out);
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

// The four links of the stencil at one site: U_x(n), U_t(n), U_x(n - x), U_t(n - t).
template <typename C> struct SiteLinks { C xf, tf, xb, tb; };

// Links of the FP32 stencil: one FP32 angle per link (the fermion boundary sign folded in as
// an added pi, wrapped to [-pi, pi]); U = cos + i sin is formed where the link is used, so
// the FP32 solver reads 4 bytes per link instead of 8.
struct LinkA32 {
    const float *A;
};
__device__ __forceinline__ float2 link_at(LinkA32 L, int i) {
    float sn, cs;
    __sincosf(L.A[i], &sn, &cs);
    return make_float2(cs, sn);
}
template <typename C> __device__ __forceinline__ C link_at(const C *__restrict__ U, int i) {
    return U[i];
}

// The links a solver of the given precision reads: FP64 complex links, or FP32 angles.
typedef const double2 *__restrict__ Link64;
template <bool MIXED> using LinkSrc = typename std::conditional<MIXED, LinkA32, Link64>::type;
template <bool MIXED, typename F> __device__ __forceinline__ LinkSrc<MIXED> link_source(const F &f) {
    if constexpr (MIXED) return LinkA32{f.A32};
    else return f.U64;
}

template <typename Src>
__device__ __forceinline__ auto site_links(Src U, const Nbr &nb, int flat, int Vtot) {
    SiteLinks<decltype(link_at(U, 0))> l;
    l.xf = link_at(U, flat);
    l.tf = link_at(U, Vtot + flat);
    l.xb = link_at(U, nb.xm);
    l.tb = link_at(U, Vtot + nb.tm);
    return l;
}

// (D a)(n) or (D^dagger a)(n) at one site, Sec. 3.  own0/own1: a(n); load(f, b0, b1)
// fetches a at flat index f.  The hopping projectors (1 -/+ sigma_mu) have rank one:
//   (1 + s sigma_1) v = (w, s w)     with w = v0 + s v1
//   (1 + s sigma_2) v = (w, s i w)   with w = v0 - s i v1
// D uses s = -1 on the forward hop and s = +1 on the backward hop; D^dagger the reverse.
template <typename T, bool DAG, typename Load>
__device__ __forceinline__ void dslash_site_links(const Nbr &nb, const SiteLinks<cplx_t<T>> &lk,
                                                  cplx_t<T> own0, cplx_t<T> own1, T mass, Load load,
                                                  cplx_t<T> &o0, cplx_t<T> &o1) {
    using C = cplx_t<T>;
    constexpr T sf = DAG ? T(1) : T(-1);  // sign on the forward hop; backward is -sf
    const C uxf = lk.xf, utf = lk.tf, uxb = lk.xb, utb = lk.tb;
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

template <typename T, bool DAG, typename Load, typename Src>
__device__ __forceinline__ void dslash_site(const Nbr &nb, int flat, int Vtot, Src U,
                                            cplx_t<T> own0, cplx_t<T> own1, T mass, Load load,
                                            cplx_t<T> &o0, cplx_t<T> &o1) {
    dslash_site_links<T, DAG>(nb, site_links(U, nb, flat, Vtot), own0, own1, mass, load, o0, o1);
}

__device__ __forceinline__ double norm2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double norm2(float2 a) {
    return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}

// Spinor access.  FP64 fields are structure-of-arrays, [s][Vtot] double2 (the public native
// layout).  The FP32 fields of the mixed-precision solver are internal and hold one float4
// (s0.re, s0.im, s1.re, s1.im) per site, so a site's spinor is a single 16-byte access.
__device__ __forceinline__ void sp_load(const double2 *__restrict__ a, int Vtot, int f, double2 &b0,
                                        double2 &b1) {
    b0 = a[f];
    b1 = a[(size_t)Vtot + f];
}
__device__ __forceinline__ void sp_load(const float4 *__restrict__ a, int, int f, float2 &b0,
                                        float2 &b1) {
    const float4 v = a[f];
    b0 = make_float2(v.x, v.y);
    b1 = make_float2(v.z, v.w);
}

__device__ __forceinline__ void sp_store(double2 *__restrict__ a, int Vtot, int f, double2 b0,
                                         double2 b1) {
    a[f] = b0;
    a[(size_t)Vtot + f] = b1;
}
__device__ __forceinline__ void sp_store(float4 *__restrict__ a, int, int f, float2 b0, float2 b1) {
    a[f] = make_float4(b0.x, b0.y, b1.x, b1.y);
}

// Write-through spinor stores, for the CG step kernels: the sc1 bit sends each 16-byte
// store through the L2 to memory at once, so an XCD's L2 holds no dirty lines of these
// fields when the kernel ends and the writeback that the end of a kernel makes (the next
// kernel reads the fields through the other XCDs' L2s) has little left to do.  On the batched
// workload this shortens the step kernels by 2-4 %.
// - The store is inline assembly: no builtin gives a global store with this bit (the
//   buffer-store builtin does, but its 32-bit offsets cannot span the largest fields).
// - A VALU write to the data registers of a store wider than 8 bytes must trail it by one
//   wait state; the compiler cannot see inside the asm, so the asm carries the wait.
// - The compiler does not count these stores as outstanding, so a barrier after them does
//   not wait for them: a kernel may use them only for fields that no other thread of it
//   reads afterwards (true of the step kernels, whose stencil reads come from LDS or from
//   fields the kernel does not write).  The end of the kernel waits for them.
// - NT adds the non-temporal bit, with which the line is not kept in the Infinity Cache.
//   That pays when the solver's fields are far larger than that cache (256 MB) and costs
//   when they fit: on single lattices and batches, an FP32 iteration is 2-4 % faster with it
//   from 16.7 M sites up, about the same at 4.2 M and 20 % slower at 1 M (the batched
//   workload, 1.6 M sites, 8 % slower); an FP64 iteration 6-8 % faster from 4.2 M up.
//   stream_fields() makes the choice.
typedef float f4v __attribute__((ext_vector_type(4)));
template <bool NT> __device__ __forceinline__ void store_wt(void *p, f4v v) {
    if constexpr (NT)
        asm volatile("global_store_dwordx4 %0, %1, off sc1 nt\n\ts_nop 1" : : "v"(p), "v"(v) : "memory");
    else
        asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 1" : : "v"(p), "v"(v) : "memory");
}
template <bool NT>
__device__ __forceinline__ void sp_store_wt(double2 *__restrict__ a, int Vtot, int f, double2 b0,
                                            double2 b1) {
    store_wt<NT>(a + f, __builtin_bit_cast(f4v, b0));
    store_wt<NT>(a + (size_t)Vtot + f, __builtin_bit_cast(f4v, b1));
}
template <bool NT>
__device__ __forceinline__ void sp_store_wt(float4 *__restrict__ a, int, int f, float2 b0, float2 b1) {
    f4v v = {b0.x, b0.y, b1.x, b1.y};
    store_wt<NT>(a + f, v);
}

// Non-temporal stores in the step kernels when the fields one iteration touches (about
// 88 B/site in FP32 with FP32 link angles, 192 B/site in FP64) exceed twice the Infinity Cache.
static bool stream_fields(const Geo &g, bool mixed) {
    const double bytes = (double)g.Vtot * (mixed ? 88.0 : 192.0);
    return bytes > 512.0 * 1024 * 1024;
}
template <bool MIXED> struct Prec;
template <> struct Prec<false> { using R = double; using S = double2; };  // S: spinor storage
template <> struct Prec<true> { using R = float; using S = float4; };

// Workgroup staging of a spinor field in LDS.  A workgroup of B threads owns the half-site
// range [w.start, w.start + B/2) of both parity planes of its chain, thread
// par * B/2 + (i - w.start) the site (par, i), so the slot of a site is its thread index.
// A stencil neighbour whose half-site index falls in the range is read from the slot; the
// others (the rows above and below the workgroup's strip) come from global memory.
template <typename C> struct LdsSpinor { C a, b; };
extern __shared__ double smem_d[];

// LDS slot of the site at flat index fl, or -1 if the workgroup does not own it.
__device__ __forceinline__ int lds_slot(const ChainInfo &ci, const BlockWork &w, int half, int fl) {
    const int loc = fl - ci.off;
    const int par = loc >= ci.Vh ? 1 : 0;
    const int k = loc - par * ci.Vh - w.start;
    return (unsigned)k < (unsigned)half ? par * half + k : -1;
}

// Loop over the sites of this workgroup; `local` is the chain-local site index.  Threads
// [0, B/2) take the even plane and [B/2, B) the odd plane at the same half-site indices.
#define SITES_LOOP                                                                \
    const int half_ = (int)blockDim.x >> 1;                                       \
    const int par_ = (int)threadIdx.x >= half_ ? 1 : 0;                           \
    for (int j_ = 0; j_ < w.spt; ++j_) {                                          \
        const int i_ = w.start + (int)threadIdx.x - par_ * half_ + j_ * half_;    \
        if (i_ >= ci.Vh) break;                                                   \
        const int local = par_ * ci.Vh + i_;
#define SITES_BEGIN                                                               \
    const BlockWork w = g.work[blockIdx.x];                                       \
    const ChainInfo ci = g.chains[w.chain];                                       \
    const int Vtot = g.Vtot;                                                      \
    (void)Vtot;                                                                   \
    SITES_LOOP
#define SITES_END }

// ================================================================ layout
__global__ void k_pack_links(Geo g, double *__restrict__ lex, double *__restrict__ nat,
                             int to_native) {
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    const size_t l = 2 * ((size_t)ci.off + s.x + (size_t)ci.Lx * s.t);
    for (int mu = 0; mu < 2; ++mu) {
        if (to_native) nat[(size_t)mu * Vtot + s.flat] = lex[l + mu];
        else lex[l + mu] = nat[(size_t)mu * Vtot + s.flat];
    }
    SITES_END
}

__global__ void k_pack_spinor(Geo g, double2 *__restrict__ lex, double2 *__restrict__ nat,
                              int to_native) {
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    const size_t l = 2 * ((size_t)ci.off + s.x + (size_t)ci.Lx * s.t);
    for (int sp = 0; sp < 2; ++sp) {
        if (to_native) nat[(size_t)sp * Vtot + s.flat] = lex[l + sp];
        else lex[l + sp] = nat[(size_t)sp * Vtot + s.flat];
    }
    SITES_END
}

void launch_pack_links(const Geo &g, double *lex, double *nat, bool to_native, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_links, dim3(g.nblocks), dim3(g.block), 0, s, g, lex, nat,
                       to_native ? 1 : 0);
}
void launch_pack_spinor(const Geo &g, double2 *lex, double2 *nat, bool to_native, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_spinor, dim3(g.nblocks), dim3(g.block), 0, s, g, lex, nat,
                       to_native ? 1 : 0);
}

// ================================================================ links
// U_mu(n) = exp(i q_mu(n)); the t-link leaving the last time slice carries the
// antiperiodic fermion boundary sign.
__global__ void k_make_links(Geo g, const double *__restrict__ q, double2 *__restrict__ U64,
                             float *__restrict__ A32) {
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    for (int mu = 0; mu < 2; ++mu) {
        const double th = q[(size_t)mu * Vtot + s.flat];
        const bool bc = mu == 1 && s.t == ci.Lt - 1;
        double sn, cs;
        sincos(th, &sn, &cs);
        if (bc) { sn = -sn; cs = -cs; }
        U64[(size_t)mu * Vtot + s.flat] = make_double2(cs, sn);
        // FP32 angle: the boundary sign as +pi, wrapped in FP64 before rounding
        if (A32) A32[(size_t)mu * Vtot + s.flat] = (float)remainder(bc ? th + M_PI : th, 2.0 * M_PI);
    }
    SITES_END
}

void launch_make_links(const Geo &g, const double *q, double2 *U64, float *A32, hipStream_t s) {
    hipLaunchKernelGGL(k_make_links, dim3(g.nblocks), dim3(g.block), 0, s, g, q, U64, A32);
}

// ================================================================ Dirac operator
// Each thread stages its own sites' input spinor in LDS; the stencil reads the neighbours
// from there when the workgroup owns them (the other parity plane at nearby half-site
// indices) and from global memory otherwise.  Outputs are stored write-through (no other
// thread of the kernel reads them), non-temporal as well when the fields are far larger than
// the Infinity Cache.
template <bool DAG, bool NT>
__global__ void k_dslash64(Geo g, const double2 *__restrict__ U, const double2 *__restrict__ in,
                           double2 *__restrict__ out) {
    LdsSpinor<double2> *lds = (LdsSpinor<double2> *)smem_d;
    const BlockWork w = g.work[blockIdx.x];
    const ChainInfo ci = g.chains[w.chain];
    const int Vtot = g.Vtot;
    const int half = (int)blockDim.x >> 1;
    const int span = half * w.spt;
    const int par = (int)threadIdx.x >= half ? 1 : 0;
    const int i0 = w.start + (int)threadIdx.x - par * half;
    for (int j = 0; j < w.spt; ++j) {
        const int i = i0 + j * half;
        if (i >= ci.Vh) break;
        const int fl = ci.off + par * ci.Vh + i;
        lds[par * span + i - w.start].a = in[fl];
        lds[par * span + i - w.start].b = in[(size_t)Vtot + fl];
    }
    __syncthreads();
    auto load = [&](int f, double2 &b0, double2 &b1) {
        const int k = lds_slot(ci, w, span, f);
        if (k >= 0) { b0 = lds[k].a; b1 = lds[k].b; }
        else { b0 = in[f]; b1 = in[(size_t)Vtot + f]; }
    };
    for (int j = 0; j < w.spt; ++j) {
        const int i = i0 + j * half;
        if (i >= ci.Vh) break;
        const Site s = decode_site(ci, par * ci.Vh + i);
        const Nbr nb = neighbours(ci, s);
        const LdsSpinor<double2> own = lds[par * span + i - w.start];
        double2 o0, o1;
        dslash_site<double, DAG>(nb, s.flat, Vtot, U, own.a, own.b, 2.0 + ci.m0, load, o0, o1);
        sp_store_wt<NT>(out, Vtot, s.flat, o0, o1);
    }
}

void launch_dslash64(const Geo &g, const double2 *U, const double2 *in, double2 *out, bool dagger,
                     hipStream_t s) {
    const size_t lds = (size_t)2 * g.block * sizeof(LdsSpinor<double2>);  // up to 2 sites per thread
    const bool nt = (double)g.Vtot * 96.0 > 512.0 * 1024 * 1024;
    if (dagger && nt) hipLaunchKernelGGL((k_dslash64<true, true>), dim3(g.nblocks), dim3(g.block), lds, s, g, U, in, out);
    else if (dagger) hipLaunchKernelGGL((k_dslash64<true, false>), dim3(g.nblocks), dim3(g.block), lds, s, g, U, in, out);
    else if (nt) hipLaunchKernelGGL((k_dslash64<false, true>), dim3(g.nblocks), dim3(g.block), lds, s, g, U, in, out);
    else hipLaunchKernelGGL((k_dslash64<false, false>), dim3(g.nblocks), dim3(g.block), lds, s, g, U, in, out);
}

// ================================================================ CG on D^dagger D
// FP64 solver: slots are plain CG iterations.  Mixed solver: slots are FP32 CG
// iterations, except that whenever the FP32 residual has dropped by delta since the last
// FP64 recomputation (or reached the target) the next slot recomputes
// r = phi - D^dagger D (x64 + x32) in FP64, folds x32 into x64 and restarts the FP32
// residual from it (reliable update); convergence is only declared on that FP64 residual.
//
// The solution update x += alpha_k p_k of iteration k is deferred to step 1 of the next
// slot, which reads p_k (as p_old) on its own sites anyway; step 2 then touches only t and
// r.  The pending alpha travels in the state: step 2 of a normal slot stores its alpha,
// step 1 of an update slot carries the pending alpha forward so that step 2 of that slot
// folds it into x64 together with x32, and a chain that stops (converged, or the final
// decision-only launch) applies it before leaving.
template <bool MIXED>
__global__ void k_cg_init(Geo g, CGFields f, double delta2) {
    double v[1] = {0.0};
    SITES_BEGIN
    const int fl = ci.off + local;
    double2 a0, a1;
    sp_load(f.phi, Vtot, fl, a0, a1);
    const double2 z = make_double2(0.0, 0.0);
    sp_store(f.x64, Vtot, fl, z, z);
    if (MIXED) {
        f.x32[fl] = make_float4(0.f, 0.f, 0.f, 0.f);
        sp_store(f.r32, Vtot, fl, make_float2((float)a0.x, (float)a0.y),
                 make_float2((float)a1.x, (float)a1.y));
    } else {
        sp_store(f.r64, Vtot, fl, a0, a1);
    }
    v[0] += norm2(a0) + norm2(a1);
    SITES_END
    write_partials<1>(v, f.p2, g.nlog, w.logical);
    if (w.logical == ci.block0 && threadIdx.x == 0) {
        CGState S = {};
        S.mode = kModeInit;
        S.delta2 = delta2;
        f.st[(size_t)g.nchains + w.chain] = S;  // parity 1: the state "before" slot 0
    }
}

// The step kernels take the tables a workgroup reads first (its work entry, the chain table,
// the CG states) and the slot as leading scalar arguments: the library is built with kernarg
// preloading, so these arrive in SGPRs at wave launch and the first table load does not wait
// for a kernarg load.  (Geo and CGFields still carry the same pointers for the rest.)
//
// Each kernel handles one work entry per workgroup, or, in the resident variant, a grid of at
// most the workgroups that fit on the GPU at once walks the list (entry b, b + grid, ...).
// SPT sites per thread: a workgroup of B threads owns the half-site range
// [start, start + SPT B/2) of both parity planes; thread t takes plane t >= B/2 and the
// half-sites start + (t mod B/2) + j B/2, j < SPT, whose LDS slot is
// plane * SPT B/2 + (t mod B/2) + j B/2.
template <bool MIXED, bool NT, int SPT>
__device__ __forceinline__ void step1_entry(const BlockWork w, const ChainInfo *__restrict__ chains,
                                            CGState *__restrict__ states, int slot, int nchains,
                                            const Geo &g, const CGFields &f, double tol2, int max_iter,
                                            const void *p_old_v, void *p_new_v, int decide_only,
                                            int sample) {
    using R = typename Prec<MIXED>::R;
    using S = typename Prec<MIXED>::S;
    using C = cplx_t<R>;
    CGState *out = states + (size_t)(slot & 1) * nchains + w.chain;
    const CGState *prev = states + (size_t)((slot + 1) & 1) * nchains + w.chain;
    // The state is read field by field in scalars (a whole-struct copy per thread would be
    // placed in LDS by the compiler), before the chain's table entry, so that both loads are
    // in flight together.
    const int p_conv = prev->converged;
    const int p_mode = prev->mode, p_iters = prev->iters, p_nupd = prev->n_updates;
    const double p_rho = prev->rho, p_rho_p = prev->rho_p, p_target = prev->target;
    const double p_phi2 = prev->phi2, p_rmax2 = prev->rmax2, delta2 = prev->delta2;
    const double p_alpha = prev->alpha;
    const ChainInfo ci = chains[w.chain];
    const int Vtot = g.Vtot;
    const bool leader = w.logical == ci.block0 && threadIdx.x == 0;
    if (p_conv) {
        if (leader) *out = *prev;
        return;
    }
    // x update still owed by the previous slot (none after the initial or an update slot)
    const double pend = p_mode == kModeNormal ? p_alpha : 0.0;
    // The operands of a normal slot on the own sites are loaded before the chain total, so
    // their latency overlaps its partial loads (they go unused in the other modes).
    const S *__restrict__ p_old = (const S *)p_old_v;
    S *__restrict__ p_new = (S *)p_new_v;
    const S *__restrict__ r;
    S *__restrict__ t;
    S *__restrict__ x;
    if constexpr (MIXED) { r = f.r32; t = f.t32; x = f.x32; }
    else { r = f.r64; t = f.t64; x = f.x64; }
    const LinkSrc<MIXED> U = link_source<MIXED>(f);
    const int half = (int)blockDim.x >> 1;
    const int span = half * SPT;
    const int par = (int)threadIdx.x >= half ? 1 : 0;
    const int i0 = w.start + (int)threadIdx.x - par * half;
    const bool first = p_mode == kModeInit;
    bool own[SPT];
    Site s[SPT];
    Nbr nb[SPT];
    SiteLinks<C> lk[SPT];
    C a0[SPT], a1[SPT], q0[SPT], q1[SPT], x0[SPT], x1[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int i = i0 + j * half;
        own[j] = i < ci.Vh;
        s[j] = Site{};
        nb[j] = Nbr{};
        lk[j] = SiteLinks<C>{};
        a0[j] = a1[j] = q0[j] = q1[j] = x0[j] = x1[j] = C{};
        if (own[j]) {
            s[j] = decode_site(ci, par * ci.Vh + i);
            nb[j] = neighbours(ci, s[j]);
            sp_load(r, Vtot, s[j].flat, a0[j], a1[j]);
            if (!first) {
                sp_load(p_old, Vtot, s[j].flat, q0[j], q1[j]);
                sp_load(x, Vtot, s[j].flat, x0[j], x1[j]);
            }
            lk[j] = site_links(U, nb[j], s[j].flat, Vtot);
        }
    }
    const double rho = chain_total(f.p2, f.fin2, ci, w.chain);
    double n_rho = rho, n_rho_p = p_rho_p, n_target = p_target, n_phi2 = p_phi2, n_rmax2 = p_rmax2;
    double n_beta = 0.0;
    int n_iters = p_iters, n_nupd = p_nupd, n_conv = 0;
    bool update = false;
    if (first) {
        n_phi2 = rho; n_target = tol2 * rho; n_rmax2 = rho; n_rho_p = rho;
        n_iters = 0; n_nupd = 0;
        n_conv = rho <= n_target ? kConverged : 0;
    } else if (p_mode == kModeUpdate) {
        n_nupd = p_nupd + 1;
        n_rmax2 = rho;
        n_conv = rho <= n_target ? kConverged : 0;
        n_beta = rho / p_rho_p;
    } else {
        n_iters = p_iters + 1;
        n_rho_p = p_rho;
        n_beta = rho / p_rho;
        if (!MIXED) n_conv = rho <= n_target ? kConverged : 0;
        else update = rho <= n_target || rho <= delta2 * n_rmax2;
    }
    // an unconverged chain stops on a non-finite residual, or at the iteration cap unless
    // this slot recomputes its FP64 residual (which decides convergence)
    if (!n_conv && !update) {
        if (!isfinite(rho)) n_conv = kStopNonFinite;
        else if (n_iters >= max_iter) n_conv = kStopMaxIter;
    }
    if (leader) {
        out->rho = n_rho; out->rho_p = n_rho_p; out->target = n_target; out->phi2 = n_phi2;
        out->rmax2 = n_rmax2; out->beta = n_beta; out->delta2 = delta2; out->iters = n_iters;
        out->converged = n_conv; out->mode = update ? kModeUpdate : kModeNormal;
        out->n_updates = n_nupd;
        out->alpha = update ? pend : 0.0;
        if (!n_conv && !decide_only) {
            // timing: the algorithmic bytes of both steps of this slot for this chain, in the
            // sampled slot's row and in the running sums over every slot
            const double b1 = ci.V * (!MIXED ? kBytesFp64Step1 : update ? kBytesUpdateStep1 : kBytesFp32Step1);
            const double b2 = ci.V * (!MIXED ? kBytesFp64Step2 : update ? kBytesUpdateStep2 : kBytesFp32Step2);
            if (sample >= 0) {
                double *row = f.samples + ((size_t)sample * g.nchains + w.chain) * 2;
                row[0] = b1;
                row[1] = b2;
            }
            if (f.all_bytes) {
                f.all_bytes[2 * w.chain] += b1;
                f.all_bytes[2 * w.chain + 1] += b2;
            }
        }
    }
    const R a_pend = (R)pend;
    if (n_conv || decide_only) {
        // the chain stops here: settle the owed x update on the own sites
        if (pend != 0.0) {
            SITES_LOOP
            const int fl = ci.off + local;
            C q0, q1, x0, x1;
            sp_load(p_old, Vtot, fl, q0, q1);
            if constexpr (MIXED) sp_load(f.x32, Vtot, fl, x0, x1);
            else sp_load(f.x64, Vtot, fl, x0, x1);
            x0.x += a_pend * q0.x; x0.y += a_pend * q0.y;
            x1.x += a_pend * q1.x; x1.y += a_pend * q1.y;
            if constexpr (MIXED) sp_store_wt<NT>(f.x32, Vtot, fl, x0, x1);
            else sp_store_wt<NT>(f.x64, Vtot, fl, x0, x1);
            SITES_END
        }
        return;
    }
    if (MIXED && update) {
        // FP64 residual recomputation, first half: t64 = D (x64 + x32 + pend p_old); p carried
        // over (step 2 of this slot folds x32 + pend p into x64).
        SITES_LOOP
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int fl, double2 &b0, double2 &b1) {
            double2 y0, y1;
            sp_load(f.x64, Vtot, fl, y0, y1);
            const float4 z = f.x32[fl];
            C q0, q1;
            sp_load(p_old, Vtot, fl, q0, q1);
            b0 = make_double2(y0.x + (double)(z.x + a_pend * q0.x), y0.y + (double)(z.y + a_pend * q0.y));
            b1 = make_double2(y1.x + (double)(z.z + a_pend * q1.x), y1.y + (double)(z.w + a_pend * q1.y));
        };
        double2 a0, a1, o0, o1;
        load(s.flat, a0, a1);
        dslash_site<double, false>(nb, s.flat, Vtot, f.U64, a0, a1, 2.0 + ci.m0, load, o0, o1);
        sp_store_wt<NT>(f.t64, Vtot, s.flat, o0, o1);
        C q0, q1;
        sp_load(p_old, Vtot, s.flat, q0, q1);
        sp_store_wt<NT>(p_new, Vtot, s.flat, q0, q1);
        SITES_END
        return;
    }
    const R beta = (R)n_beta;
    // Own sites: x += pend p_old (deferred from the previous slot), p_new = r + beta p_old,
    // staged in LDS for the neighbours inside the workgroup; t = D p_new.
    LdsSpinor<C> *lds = (LdsSpinor<C> *)smem_d;
    auto direction = [&](int fl, C &b0, C &b1) {
        sp_load(r, Vtot, fl, b0, b1);
        if (!first) {
            C c0, c1;
            sp_load(p_old, Vtot, fl, c0, c1);
            b0 = cmake<C>(b0.x + beta * c0.x, b0.y + beta * c0.y);
            b1 = cmake<C>(b1.x + beta * c1.x, b1.y + beta * c1.y);
        }
    };
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        if (!own[j]) continue;
        if (!first) {
            x0[j].x += a_pend * q0[j].x; x0[j].y += a_pend * q0[j].y;
            x1[j].x += a_pend * q1[j].x; x1[j].y += a_pend * q1[j].y;
            sp_store_wt<NT>(x, Vtot, s[j].flat, x0[j], x1[j]);
            a0[j] = cmake<C>(a0[j].x + beta * q0[j].x, a0[j].y + beta * q0[j].y);
            a1[j] = cmake<C>(a1[j].x + beta * q1[j].x, a1[j].y + beta * q1[j].y);
        }
        sp_store_wt<NT>(p_new, Vtot, s[j].flat, a0[j], a1[j]);
        const int k = par * span + (int)threadIdx.x - par * half + j * half;
        lds[k].a = a0[j];
        lds[k].b = a1[j];
    }
    __syncthreads();
    double v[1] = {0.0};
    auto load = [&](int fl, C &b0, C &b1) {
        const int k = lds_slot(ci, w, span, fl);
        if (k >= 0) { b0 = lds[k].a; b1 = lds[k].b; }
        else direction(fl, b0, b1);
    };
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        if (!own[j]) continue;
        C o0, o1;
        dslash_site_links<R, false>(nb[j], lk[j], a0[j], a1[j], (R)(2.0 + ci.m0), load, o0, o1);
        sp_store_wt<NT>(t, Vtot, s[j].flat, o0, o1);
        v[0] += norm2(o0) + norm2(o1);
    }
    write_partials<1>(v, f.p1, g.nlog, w.logical);
}

template <bool MIXED, bool NT, int SPT>
__device__ __forceinline__ void step2_entry(const BlockWork w, const ChainInfo *__restrict__ chains,
                                            CGState *__restrict__ states, int slot, int nchains,
                                            const Geo &g, const CGFields &f, const void *p_new_v) {
    using R = typename Prec<MIXED>::R;
    using S = typename Prec<MIXED>::S;
    using C = cplx_t<R>;
    CGState *st = states + (size_t)(slot & 1) * nchains + w.chain;
    // the state's fields before the chain's table entry, so that both loads are in flight
    // together
    const int s_conv = st->converged, mode = st->mode;
    const double s_rho = st->rho;
    const ChainInfo ci = chains[w.chain];
    const int Vtot = g.Vtot;
    // An empty asm that reads the table fields: it keeps the compiler from sinking the table
    // load below the early return, so the state and the table are waited for together (one
    // memory latency instead of two before the site loads).  Step 1 measured faster without it.
    asm volatile("" : : "s"(s_rho), "s"(ci.off), "s"(ci.Vh), "s"(ci.block0), "s"(ci.nblocks),
                 "s"(ci.m0));
    if (s_conv) return;
    double v[1] = {0.0};
    if (MIXED && mode == kModeUpdate) {
        // second half: r64 = phi - D^dagger t64; x64 += x32 + pend p; x32 = 0; r32 = r64.
        const float a_pend = (float)st->alpha;
        const float4 *__restrict__ p = (const float4 *)p_new_v;
        SITES_LOOP
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int fl, double2 &b0, double2 &b1) { sp_load(f.t64, Vtot, fl, b0, b1); };
        double2 a0, a1, t0, t1;
        load(s.flat, t0, t1);
        dslash_site<double, true>(nb, s.flat, Vtot, f.U64, t0, t1, 2.0 + ci.m0, load, a0, a1);
        double2 h0, h1, x0, x1;
        sp_load(f.phi, Vtot, s.flat, h0, h1);
        sp_load(f.x64, Vtot, s.flat, x0, x1);
        const float4 z = f.x32[s.flat];
        const float4 q = p[s.flat];
        const double2 r0 = make_double2(h0.x - a0.x, h0.y - a0.y);
        const double2 r1 = make_double2(h1.x - a1.x, h1.y - a1.y);
        sp_store_wt<NT>(f.x64, Vtot, s.flat,
                 make_double2(x0.x + (double)(z.x + a_pend * q.x), x0.y + (double)(z.y + a_pend * q.y)),
                 make_double2(x1.x + (double)(z.z + a_pend * q.z), x1.y + (double)(z.w + a_pend * q.w)));
        f.x32[s.flat] = make_float4(0.f, 0.f, 0.f, 0.f);
        sp_store_wt<NT>(f.r32, Vtot, s.flat, make_float2((float)r0.x, (float)r0.y),
                 make_float2((float)r1.x, (float)r1.y));
        v[0] += norm2(r0) + norm2(r1);
        SITES_END
        write_partials<1>(v, f.p2, g.nlog, w.logical);
        return;
    }
    const S *__restrict__ t;
    S *__restrict__ r;
    if constexpr (MIXED) { t = f.t32; r = f.r32; }
    else { t = f.t64; r = f.r64; }
    const LinkSrc<MIXED> U = link_source<MIXED>(f);
    // The own sites' t, r and links are loaded before the chain total, so their latency
    // overlaps its partial loads.  t is staged in LDS for the neighbours inside the
    // workgroup.
    LdsSpinor<C> *lds = (LdsSpinor<C> *)smem_d;
    const int half = (int)blockDim.x >> 1;
    const int span = half * SPT;
    const int par = (int)threadIdx.x >= half ? 1 : 0;
    const int i0 = w.start + (int)threadIdx.x - par * half;
    bool own[SPT];
    Site s[SPT];
    Nbr nb[SPT];
    SiteLinks<C> lk[SPT];
    C t0[SPT], t1[SPT], r0[SPT], r1[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int i = i0 + j * half;
        own[j] = i < ci.Vh;
        s[j] = Site{};
        nb[j] = Nbr{};
        lk[j] = SiteLinks<C>{};
        t0[j] = t1[j] = r0[j] = r1[j] = C{};
        if (own[j]) {
            s[j] = decode_site(ci, par * ci.Vh + i);
            nb[j] = neighbours(ci, s[j]);
            sp_load(t, Vtot, s[j].flat, t0[j], t1[j]);
            sp_load(r, Vtot, s[j].flat, r0[j], r1[j]);
            lk[j] = site_links(U, nb[j], s[j].flat, Vtot);
            const int k = par * span + (int)threadIdx.x - par * half + j * half;
            lds[k].a = t0[j];
            lds[k].b = t1[j];
        }
    }
    const double pAp = chain_total(f.p1, f.fin1, ci, w.chain);
    const double alpha_d = s_rho / pAp;
    if (w.logical == ci.block0 && threadIdx.x == 0) st->alpha = alpha_d;  // owed to x (next slot)
    const R alpha = (R)alpha_d;
    __syncthreads();
    auto load = [&](int fl, C &b0, C &b1) {
        const int k = lds_slot(ci, w, span, fl);
        if (k >= 0) { b0 = lds[k].a; b1 = lds[k].b; }
        else sp_load(t, Vtot, fl, b0, b1);
    };
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        if (!own[j]) continue;
        C a0, a1;
        dslash_site_links<R, true>(nb[j], lk[j], t0[j], t1[j], (R)(2.0 + ci.m0), load, a0, a1);
        r0[j].x -= alpha * a0.x; r0[j].y -= alpha * a0.y;
        r1[j].x -= alpha * a1.x; r1[j].y -= alpha * a1.y;
        sp_store_wt<NT>(r, Vtot, s[j].flat, r0[j], r1[j]);
        v[0] += norm2(r0[j]) + norm2(r1[j]);
    }
    write_partials<1>(v, f.p2, g.nlog, w.logical);
}

// The entry loop of the resident variant: a barrier between entries, so that no thread
// rewrites LDS (the staged spinors, the partial sums) while another still reads the previous
// entry's.
// With f.active set (captured iteration chunks), the entry count comes from the device.
#define STEP_ENTRIES(RES, BODY)                                                          \
    const int n_entries = f.active ? *f.active : g.nblocks;                              \
    if constexpr (RES) {                                                                 \
        for (int b = blockIdx.x; b < n_entries; b += gridDim.x) {                        \
            if (b != (int)blockIdx.x) __syncthreads();                                   \
            BODY(work[b]);                                                               \
        }                                                                                \
    } else if ((int)blockIdx.x < n_entries) {                                            \
        BODY(work[blockIdx.x]);                                                          \
    }

template <bool MIXED, bool NT, int SPT, bool RES>
__global__ void k_cg_step1(const BlockWork *__restrict__ work, const ChainInfo *__restrict__ chains,
                           CGState *__restrict__ states, int slot, int nchains, Geo g, CGFields f,
                           double tol2, int max_iter, const void *p_old_v, void *p_new_v,
                           int decide_only, int sample) {
#define BODY1(W) step1_entry<MIXED, NT, SPT>(W, chains, states, slot, nchains, g, f, tol2, max_iter, \
                                             p_old_v, p_new_v, decide_only, sample)
    STEP_ENTRIES(RES, BODY1)
#undef BODY1
}

// The same with at most 64 VGPRs (8 waves per SIMD): the occupancy variant.
template <bool MIXED, bool NT>
__global__ void __attribute__((amdgpu_waves_per_eu(8)))
k_cg_step1_w8(const BlockWork *__restrict__ work, const ChainInfo *__restrict__ chains,
              CGState *__restrict__ states, int slot, int nchains, Geo g, CGFields f, double tol2,
              int max_iter, const void *p_old_v, void *p_new_v, int decide_only, int sample) {
#define BODY1(W) step1_entry<MIXED, NT, 1>(W, chains, states, slot, nchains, g, f, tol2, max_iter, \
                                           p_old_v, p_new_v, decide_only, sample)
    STEP_ENTRIES(false, BODY1)
#undef BODY1
}

template <bool MIXED, bool NT, int SPT, bool RES>
__global__ void k_cg_step2(const BlockWork *__restrict__ work, const ChainInfo *__restrict__ chains,
                           CGState *__restrict__ states, int slot, int nchains, Geo g, CGFields f,
                           const void *p_new_v) {
#define BODY2(W) step2_entry<MIXED, NT, SPT>(W, chains, states, slot, nchains, g, f, p_new_v)
    STEP_ENTRIES(RES, BODY2)
#undef BODY2
}

template <bool MIXED, bool NT>
__global__ void __attribute__((amdgpu_waves_per_eu(8)))
k_cg_step2_w8(const BlockWork *__restrict__ work, const ChainInfo *__restrict__ chains,
              CGState *__restrict__ states, int slot, int nchains, Geo g, CGFields f,
              const void *p_new_v) {
#define BODY2(W) step2_entry<MIXED, NT, 1>(W, chains, states, slot, nchains, g, f, p_new_v)
    STEP_ENTRIES(false, BODY2)
#undef BODY2
}

__global__ void k_cg_finish_mixed(Geo g, CGFields f) {
    SITES_BEGIN
    const int fl = ci.off + local;
    double2 x0, x1;
    sp_load(f.x64, Vtot, fl, x0, x1);
    const float4 z = f.x32[fl];
    sp_store(f.x64, Vtot, fl, make_double2(x0.x + (double)z.x, x0.y + (double)z.y),
             make_double2(x1.x + (double)z.z, x1.y + (double)z.w));
    f.x32[fl] = make_float4(0.f, 0.f, 0.f, 0.f);
    SITES_END
}

void launch_cg_init(const Geo &g, const CGFields &f, bool mixed, double delta, hipStream_t s) {
    if (mixed) hipLaunchKernelGGL(k_cg_init<true>, dim3(g.nblocks), dim3(g.block), 0, s, g, f, delta * delta);
    else hipLaunchKernelGGL(k_cg_init<false>, dim3(g.nblocks), dim3(g.block), 0, s, g, f, delta * delta);
}

// A launch whose start and end are stamped into ev0 and ev1 by the dispatch itself (no
// marker packets around it), or a plain launch when ev0 is null.
template <typename K, typename... A>
static void launch_stamped(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1, A... args) {
    if (ev0) hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, ev0, ev1, 0u, args...);
    else hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

int step_variant_spt(int variant) { return variant == kStepTwoSites ? 2 : 1; }

// Workgroups of `kernel` resident on the whole GPU at once with `block` threads and `lds`
// bytes of dynamic LDS (cached per kernel, size and device).
static int resident_workgroups(const void *kernel, int block, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 1 << 30;
    }
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(kernel, block, lds, dev);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per_cu < 1 || cus < 1) {
        (void)hipGetLastError();
        per_cu = 1;
        cus = 256;
    }
    return cache[key] = per_cu * cus;
}

template <bool MIXED, bool NT>
static void launch_step1_inst(const Geo &g, const CGFields &f, int variant, int slot, double tol,
                              int max_iter, const void *p_old, void *p_new, bool decide_only,
                              int sample, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    using C = cplx_t<typename Prec<MIXED>::R>;
    const size_t lds = (size_t)g.block * step_variant_spt(variant) * sizeof(LdsSpinor<C>);
    const int dec = decide_only ? 1 : 0;
#define ARGS1 s, ev0, ev1, g.work, g.chains, f.st, slot, g.nchains, g, f, tol * tol, max_iter, p_old, \
              p_new, dec, sample
    switch (variant) {
    case kStepTwoSites:
        launch_stamped(k_cg_step1<MIXED, NT, 2, false>, dim3(g.nblocks), dim3(g.block), lds, ARGS1);
        break;
    case kStepResident: {
        const void *k = (const void *)k_cg_step1<MIXED, NT, 1, true>;
        const int grid = std::min(g.nblocks, resident_workgroups(k, g.block, lds));
        launch_stamped(k_cg_step1<MIXED, NT, 1, true>, dim3(grid), dim3(g.block), lds, ARGS1);
        break;
    }
    case kStepWaves8:
        launch_stamped(k_cg_step1_w8<MIXED, NT>, dim3(g.nblocks), dim3(g.block), lds, ARGS1);
        break;
    default:
        launch_stamped(k_cg_step1<MIXED, NT, 1, false>, dim3(g.nblocks), dim3(g.block), lds, ARGS1);
    }
#undef ARGS1
}

void launch_cg_step1(const Geo &g, const CGFields &f, bool mixed, int variant, int slot, double tol,
                     int max_iter, const void *p_old, void *p_new, bool decide_only, int sample,
                     hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (g.nblocks <= 0) return;
    const bool nt = stream_fields(g, mixed);
    if (mixed && nt)
        launch_step1_inst<true, true>(g, f, variant, slot, tol, max_iter, p_old, p_new, decide_only, sample, s, ev0, ev1);
    else if (mixed)
        launch_step1_inst<true, false>(g, f, variant, slot, tol, max_iter, p_old, p_new, decide_only, sample, s, ev0, ev1);
    else if (nt)
        launch_step1_inst<false, true>(g, f, variant, slot, tol, max_iter, p_old, p_new, decide_only, sample, s, ev0, ev1);
    else
        launch_step1_inst<false, false>(g, f, variant, slot, tol, max_iter, p_old, p_new, decide_only, sample, s, ev0, ev1);
}

// One workgroup per sampled slot: the sum over chains of its byte row, which is then zeroed
// for the next solve.
__global__ void k_sample_sums(double *__restrict__ samples, int nchains, double *__restrict__ sums) {
    double v[2] = {0.0, 0.0};
    double *row = samples + (size_t)blockIdx.x * nchains * 2;
    for (int c = threadIdx.x; c < nchains; c += blockDim.x) {
        v[0] += row[2 * c];
        v[1] += row[2 * c + 1];
        row[2 * c] = 0.0;
        row[2 * c + 1] = 0.0;
    }
    block_sum_all<2>(v);
    if (threadIdx.x == 0) {
        sums[2 * blockIdx.x] = v[0];
        sums[2 * blockIdx.x + 1] = v[1];
    }
}

void launch_sample_sums(double *samples, int n, int nchains, double *sums, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_sample_sums, dim3(n), dim3(256), 0, s, samples, nchains, sums);
}

template <bool MIXED, bool NT>
static void launch_step2_inst(const Geo &g, const CGFields &f, int variant, int slot, const void *p_new,
                              hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    using C = cplx_t<typename Prec<MIXED>::R>;
    const size_t lds = (size_t)g.block * step_variant_spt(variant) * sizeof(LdsSpinor<C>);
#define ARGS2 s, ev0, ev1, g.work, g.chains, f.st, slot, g.nchains, g, f, p_new
    switch (variant) {
    case kStepTwoSites:
        launch_stamped(k_cg_step2<MIXED, NT, 2, false>, dim3(g.nblocks), dim3(g.block), lds, ARGS2);
        break;
    case kStepResident: {
        const void *k = (const void *)k_cg_step2<MIXED, NT, 1, true>;
        const int grid = std::min(g.nblocks, resident_workgroups(k, g.block, lds));
        launch_stamped(k_cg_step2<MIXED, NT, 1, true>, dim3(grid), dim3(g.block), lds, ARGS2);
        break;
    }
    case kStepWaves8:
        launch_stamped(k_cg_step2_w8<MIXED, NT>, dim3(g.nblocks), dim3(g.block), lds, ARGS2);
        break;
    default:
        launch_stamped(k_cg_step2<MIXED, NT, 1, false>, dim3(g.nblocks), dim3(g.block), lds, ARGS2);
    }
#undef ARGS2
}

void launch_cg_step2(const Geo &g, const CGFields &f, bool mixed, int variant, int slot,
                     const void *p_new, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (g.nblocks <= 0) return;
    const bool nt = stream_fields(g, mixed);
    if (mixed && nt) launch_step2_inst<true, true>(g, f, variant, slot, p_new, s, ev0, ev1);
    else if (mixed) launch_step2_inst<true, false>(g, f, variant, slot, p_new, s, ev0, ev1);
    else if (nt) launch_step2_inst<false, true>(g, f, variant, slot, p_new, s, ev0, ev1);
    else launch_step2_inst<false, false>(g, f, variant, slot, p_new, s, ev0, ev1);
}

void launch_cg_finish_mixed(const Geo &g, const CGFields &f, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_finish_mixed, dim3(g.nblocks), dim3(g.block), 0, s, g, f);
}

// ---------------------------------------------------------------- fused CG iteration
// One kernel per CG iteration, for chains whose workgroups own whole lattice rows: a
// workgroup of B threads owns rows [t0, t0 + nr) of both parity planes (nr = (B/2) / (Lx/2)),
// or the whole chain.  The standard CG recurrences are regrouped so that each iteration
// needs one grid-wide reduction point, which the kernel boundary provides: slot k
// receives the dot products of slot k-1 (||t||^2 = <p, A p>, ||r||^2, Re<r, s>, ||s||^2 with
// t = D p and s = A p = D^dagger t), takes the step alpha = ||r||^2 / ||t||^2 of the previous
// direction (r -= alpha s, x += alpha p), predicts ||r_new||^2 = ||r||^2 - 2 alpha Re<r, s>
// + alpha^2 ||s||^2 for beta, forms p = r + beta p, and applies A to it.  A needs p two rows
// beyond the own rows: those rows are recomputed from the previous r, s, p (read, never the
// same slot's output of another workgroup), staged with the own rows in LDS, and t is formed
// on the own rows and one row beyond.  r, s and p are double-buffered (buf in the state);
// x is only touched by its owner.

// The element-wise CG step on one site: r_new = r - a s, p_new = r_new + b p.
template <typename C, typename R>
__device__ __forceinline__ void cg_advance(C r0, C r1, C s0, C s1, C q0, C q1, R a, R b, C &rn0,
                                           C &rn1, C &pn0, C &pn1) {
    rn0 = cmake<C>(r0.x - a * s0.x, r0.y - a * s0.y);
    rn1 = cmake<C>(r1.x - a * s1.x, r1.y - a * s1.y);
    pn0 = cmake<C>(rn0.x + b * q0.x, rn0.y + b * q0.y);
    pn1 = cmake<C>(rn1.x + b * q1.x, rn1.y + b * q1.y);
}

__device__ __forceinline__ double dot_re(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }
__device__ __forceinline__ double dot_re(float2 a, float2 b) {
    return (double)a.x * (double)b.x + (double)a.y * (double)b.y;
}

// Chain total of one partial row (chains of at most kMaxChainBlocks workgroups), identical in
// every wavefront of the chain.
__device__ __forceinline__ double chain_sum(const double *__restrict__ row, const ChainInfo &ci) {
    double a = 0.0;
    for (int j = (int)(threadIdx.x & 63); j < ci.nblocks; j += 64) a += row[ci.block0 + j];
    return wave_sum(a);
}

bool cg_iter_eligible(const ChainInfo &ci, int block, int *lds_entries) {
    const int half = block / 2;
    if (ci.nblocks > kMaxChainBlocks) return false;
    if (ci.Vh <= half) {  // the whole chain in one workgroup: no halo rows
        *lds_entries = 4 * ci.Vh;
        return true;
    }
    if (half % ci.hx) return false;
    const int nr = half / ci.hx;
    if (ci.Lt < nr + 4) return false;  // the halo rows would wrap onto the own rows
    *lds_entries = 2 * ci.hx * ((nr + 4) + (nr + 2));
    return true;
}

size_t cg_iter_lds_bytes(int entries, bool mixed) {
    return (size_t)entries * (mixed ? sizeof(LdsSpinor<float2>) : sizeof(LdsSpinor<double2>));
}

template <bool MIXED>
__global__ void k_cg_iter(Geo g, CGIterFields f, int slot, double tol2, int decide_only, int sample) {
    using R = typename Prec<MIXED>::R;
    using S = typename Prec<MIXED>::S;
    using C = cplx_t<R>;
    const BlockWork w = g.work[blockIdx.x];
    const ChainInfo ci = g.chains[w.chain];
    const int Vtot = g.Vtot;
    const bool leader = w.logical == ci.block0 && threadIdx.x == 0;
    CGState *out = f.st + (size_t)(slot & 1) * g.nchains + w.chain;
    const CGState *prev = f.st + (size_t)((slot + 1) & 1) * g.nchains + w.chain;
    if (prev->converged) {
        if (leader) *out = *prev;
        return;
    }
    const int p_mode = prev->mode, p_iters = prev->iters, p_nupd = prev->n_updates, buf = prev->buf;
    const double p_target = prev->target, p_phi2 = prev->phi2, p_rmax2 = prev->rmax2;
    const double delta2 = prev->delta2, p_t2 = prev->t2, p_s2 = prev->s2;
    const bool first = p_mode == kModeInit;

    const S *__restrict__ r_old = (const S *)f.r[buf];
    const S *__restrict__ s_old = (const S *)f.s[buf];
    const S *__restrict__ p_old = (const S *)f.p[buf];
    S *__restrict__ x;
    if constexpr (MIXED) x = f.x32;
    else x = f.x64;
    const LinkSrc<MIXED> U = link_source<MIXED>(f);
    const int hx = ci.hx, Lx = ci.Lx, Lt = ci.Lt, Vh = ci.Vh;
    const int half = (int)blockDim.x >> 1;
    const int par = (int)threadIdx.x >= half ? 1 : 0;
    const int i = w.start + (int)threadIdx.x - par * half;
    const bool own = i < Vh;
    auto links_at = [&](int P, int t, int xh) {
        const int xs = 2 * xh + ((P ^ t) & 1);
        const int xm = xs == 0 ? Lx - 1 : xs - 1, tm = t == 0 ? Lt - 1 : t - 1;
        const int fl = ci.off + P * Vh + t * hx + xh;
        SiteLinks<C> l;
        l.xf = link_at(U, fl);
        l.tf = link_at(U, Vtot + fl);
        l.xb = link_at(U, ci.off + (1 - P) * Vh + t * hx + (xm >> 1));
        l.tb = link_at(U, Vtot + ci.off + (1 - P) * Vh + tm * hx + xh);
        return l;
    };
    // own site and its operands, loaded before the chain totals
    const int ot = i / hx, oxh = i - ot * hx;  // own row and column
    const int flat = ci.off + par * Vh + i;
    SiteLinks<C> lk = {};
    C r0 = {}, r1 = {}, z0 = {}, z1 = {}, q0 = {}, q1 = {};
    if (own) {
        sp_load(r_old, Vtot, flat, r0, r1);
        if (!first) {
            sp_load(s_old, Vtot, flat, z0, z1);
            sp_load(p_old, Vtot, flat, q0, q1);
        }
        lk = links_at(par, ot, oxh);
    }
    const double *Qp = f.Q + (size_t)(((slot + 1) & 1) * 4) * g.nlog;
    double *Qc = f.Q + (size_t)((slot & 1) * 4) * g.nlog;
    const double ta = chain_sum(Qp, ci), tb = chain_sum(Qp + g.nlog, ci);
    const double tc = chain_sum(Qp + 2 * g.nlog, ci), td = chain_sum(Qp + 3 * g.nlog, ci);

    // decision for this slot
    int n_mode = kModeNormal, n_iters = p_iters, n_nupd = p_nupd, n_conv = 0, n_buf = buf;
    double n_target = p_target, n_phi2 = p_phi2, n_rmax2 = p_rmax2, n_t2 = p_t2, n_s2 = p_s2;
    double alpha = 0.0, beta = 0.0;
    if (first) {  // tb = ||phi||^2 from the initial kernel; p = r
        n_phi2 = tb; n_target = tol2 * tb; n_rmax2 = tb; n_iters = 0; n_nupd = 0;
        n_conv = tb <= n_target ? kConverged : !isfinite(tb) ? kStopNonFinite : 0;
        n_buf = buf ^ 1;
    } else if (p_mode == kModeUpdate) {
        n_mode = kModeUpdate2;
    } else {
        double A = ta, D2 = td;
        if (p_mode == kModeUpdate2) {  // tb, tc: the recomputed residual against the last s
            n_nupd = p_nupd + 1;
            n_rmax2 = tb;
            A = p_t2;
            D2 = p_s2;
            n_conv = tb <= n_target ? kConverged : 0;
        } else if (!MIXED) {
            n_conv = tb <= n_target ? kConverged : 0;
        } else if (tb <= n_target || tb <= delta2 * n_rmax2) {
            n_mode = kModeUpdate;
            n_t2 = ta;
            n_s2 = td;
        }
        if (!n_conv && n_mode == kModeNormal && !isfinite(tb)) n_conv = kStopNonFinite;
        if (!n_conv && n_mode == kModeNormal) {
            alpha = tb / A;
            beta = (tb - 2.0 * alpha * tc + alpha * alpha * D2) / tb;
            if (!decide_only) {  // the step is taken by this slot
                n_iters = p_iters + 1;
                n_buf = buf ^ 1;
            }
        }
    }
    if (leader) {
        out->rho = tb; out->rho_p = 0.0; out->target = n_target; out->phi2 = n_phi2;
        out->rmax2 = n_rmax2; out->beta = beta; out->delta2 = delta2; out->alpha = alpha;
        out->t2 = n_t2; out->s2 = n_s2; out->iters = n_iters; out->converged = n_conv;
        out->mode = n_mode; out->n_updates = n_nupd; out->buf = n_buf;
        if (sample >= 0 && !n_conv && !decide_only) {
            double *row = f.samples + ((size_t)sample * g.nchains + w.chain) * 2;
            row[0] = ci.V * (n_mode == kModeUpdate ? kBytesIterUpdate1
                             : n_mode == kModeUpdate2 ? kBytesIterUpdate2
                             : MIXED ? kBytesIterFp32 : kBytesIterFp64);
            row[1] = 0.0;
        }
    }
    if (n_conv || decide_only) return;

    if (MIXED && n_mode == kModeUpdate) {
        // residual recomputation, first slot: t64 = D (x64 + x32)
        if (own) {
            const Site s = decode_site(ci, par * Vh + i);
            const Nbr nb = neighbours(ci, s);
            auto load = [&](int fl, double2 &b0, double2 &b1) {
                double2 y0, y1;
                sp_load(f.x64, Vtot, fl, y0, y1);
                const float4 zz = f.x32[fl];
                b0 = make_double2(y0.x + (double)zz.x, y0.y + (double)zz.y);
                b1 = make_double2(y1.x + (double)zz.z, y1.y + (double)zz.w);
            };
            double2 a0, a1, o0, o1;
            load(s.flat, a0, a1);
            dslash_site<double, false>(nb, s.flat, Vtot, f.U64, a0, a1, 2.0 + ci.m0, load, o0, o1);
            sp_store(f.t64, Vtot, s.flat, o0, o1);
        }
        return;
    }
    if (MIXED && n_mode == kModeUpdate2) {
        // second slot: r = phi - D^dagger t64 in FP64, x64 += x32, x32 = 0, r (FP32) in place;
        // partials ||r||^2 and Re<r, s> against the unchanged s of the last direction
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (own) {
            const Site s = decode_site(ci, par * Vh + i);
            const Nbr nb = neighbours(ci, s);
            auto load = [&](int fl, double2 &b0, double2 &b1) { sp_load(f.t64, Vtot, fl, b0, b1); };
            double2 t0, t1, a0, a1;
            load(s.flat, t0, t1);
            dslash_site<double, true>(nb, s.flat, Vtot, f.U64, t0, t1, 2.0 + ci.m0, load, a0, a1);
            double2 h0, h1, y0, y1;
            sp_load(f.phi, Vtot, s.flat, h0, h1);
            sp_load(f.x64, Vtot, s.flat, y0, y1);
            const float4 zz = f.x32[s.flat];
            const double2 e0 = make_double2(h0.x - a0.x, h0.y - a0.y);
            const double2 e1 = make_double2(h1.x - a1.x, h1.y - a1.y);
            sp_store(f.x64, Vtot, s.flat, make_double2(y0.x + (double)zz.x, y0.y + (double)zz.y),
                     make_double2(y1.x + (double)zz.z, y1.y + (double)zz.w));
            f.x32[s.flat] = make_float4(0.f, 0.f, 0.f, 0.f);
            const C e0f = cmake<C>((R)e0.x, (R)e0.y), e1f = cmake<C>((R)e1.x, (R)e1.y);
            sp_store((S *)f.r[buf], Vtot, s.flat, e0f, e1f);
            v[1] = norm2(e0) + norm2(e1);
            v[2] = dot_re(e0f, z0) + dot_re(e1f, z1);
        }
        write_partials<4>(v, Qc, g.nlog, w.logical);
        return;
    }

    // normal slot
    S *__restrict__ r_new = (S *)f.r[buf ^ 1];
    S *__restrict__ s_new = (S *)f.s[buf ^ 1];
    S *__restrict__ p_new = (S *)f.p[buf ^ 1];
    const R ra = (R)alpha, rb = (R)beta;
    const bool whole = ci.nblocks == 1;
    const int t0 = w.start / hx;
    const int nr = whole ? Lt : min(half, Vh - w.start) / hx;
    const int Hp = whole ? 0 : 2, Ht = whole ? 0 : 1;
    const int np = nr + 2 * Hp, nt = nr + 2 * Ht;
    LdsSpinor<C> *lp = (LdsSpinor<C> *)smem_d;  // [2][np][hx]: p on rows t0 - Hp ...
    LdsSpinor<C> *lt = lp + 2 * np * hx;        // [2][nt][hx]: t on rows t0 - Ht ...
    auto wslot = [&](int P, int wr, int rows, int xh) { return (P * rows + wr) * hx + xh; };
    // window slots of the stencil neighbours of the site (P, chain row t, xh), whose row
    // sits at row wr of a window of `rows` rows
    auto wnbr = [&](int P, int t, int xh, int wr, int rows) {
        const int xs = 2 * xh + ((P ^ t) & 1);
        const int xp = xs + 1 == Lx ? 0 : xs + 1, xm = xs == 0 ? Lx - 1 : xs - 1;
        int up = wr + 1, dn = wr - 1;
        if (whole) {
            if (up == Lt) up = 0;
            if (dn < 0) dn = Lt - 1;
        }
        Nbr n;
        n.xp = wslot(1 - P, wr, rows, xp >> 1);
        n.xm = wslot(1 - P, wr, rows, xm >> 1);
        n.tp = wslot(1 - P, up, rows, xh);
        n.tm = wslot(1 - P, dn, rows, xh);
        return n;
    };
    C rn0 = {}, rn1 = {}, pn0 = {}, pn1 = {};
    if (own) {
        cg_advance(r0, r1, z0, z1, q0, q1, ra, rb, rn0, rn1, pn0, pn1);
        if (!first) {
            C x0, x1;
            sp_load(x, Vtot, flat, x0, x1);
            x0.x += ra * q0.x; x0.y += ra * q0.y;
            x1.x += ra * q1.x; x1.y += ra * q1.y;
            sp_store(x, Vtot, flat, x0, x1);
        }
        sp_store(r_new, Vtot, flat, rn0, rn1);
        sp_store(p_new, Vtot, flat, pn0, pn1);
        const int k = wslot(par, ot - t0 + Hp, np, oxh);
        lp[k].a = pn0;
        lp[k].b = pn1;
    }
    if (!whole) {
        // p on the two rows below and above the own rows, from the previous r, s, p
#pragma unroll 1
        for (int h = threadIdx.x; h < 8 * hx; h += blockDim.x) {
            const int P = h / (4 * hx), rem = h - P * 4 * hx, hr = rem / hx, hxh = rem - hr * hx;
            int row = hr < 2 ? t0 - 2 + hr : t0 + nr + hr - 2;
            row = row < 0 ? row + Lt : (row >= Lt ? row - Lt : row);
            const int fl = ci.off + P * Vh + row * hx + hxh;
            C hr0, hr1, hs0 = {}, hs1 = {}, hq0 = {}, hq1 = {}, a0, a1, b0, b1;
            sp_load(r_old, Vtot, fl, hr0, hr1);
            if (!first) {
                sp_load(s_old, Vtot, fl, hs0, hs1);
                sp_load(p_old, Vtot, fl, hq0, hq1);
            }
            cg_advance(hr0, hr1, hs0, hs1, hq0, hq1, ra, rb, a0, a1, b0, b1);
            const int k = wslot(P, hr < 2 ? hr : nr + hr, np, hxh);
            lp[k].a = b0;
            lp[k].b = b1;
        }
    }
    __syncthreads();
    // t = D p on the own rows and one row beyond
    const R mass = (R)(2.0 + ci.m0);
    auto ld_p = [&](int k, C &b0, C &b1) { b0 = lp[k].a; b1 = lp[k].b; };
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    C tn0 = {}, tn1 = {};
    if (own) {
        const int wt = ot - t0 + Ht;
        dslash_site_links<R, false>(wnbr(par, ot, oxh, wt + Hp - Ht, np), lk, pn0, pn1, mass, ld_p,
                                    tn0, tn1);
        const int k = wslot(par, wt, nt, oxh);
        lt[k].a = tn0;
        lt[k].b = tn1;
        v[0] = norm2(tn0) + norm2(tn1);
    }
    if (!whole) {
#pragma unroll 1
        for (int h = threadIdx.x; h < 4 * hx; h += blockDim.x) {
            const int P = h / (2 * hx), rem = h - P * 2 * hx, hr = rem / hx, hxh = rem - hr * hx;
            int row = hr == 0 ? t0 - 1 : t0 + nr;
            row = row < 0 ? row + Lt : (row >= Lt ? row - Lt : row);
            const int wt = hr == 0 ? 0 : nr + 1, wp = wt + 1;
            C a0, a1, o0, o1;
            ld_p(wslot(P, wp, np, hxh), a0, a1);
            dslash_site_links<R, false>(wnbr(P, row, hxh, wp, np), links_at(P, row, hxh), a0, a1,
                                        mass, ld_p, o0, o1);
            const int k = wslot(P, wt, nt, hxh);
            lt[k].a = o0;
            lt[k].b = o1;
        }
    }
    __syncthreads();
    // s = D^dagger t on the own rows
    if (own) {
        auto ld_t = [&](int k, C &b0, C &b1) { b0 = lt[k].a; b1 = lt[k].b; };
        const int wt = ot - t0 + Ht;
        C sn0, sn1;
        dslash_site_links<R, true>(wnbr(par, ot, oxh, wt, nt), lk, tn0, tn1, mass, ld_t, sn0, sn1);
        sp_store(s_new, Vtot, flat, sn0, sn1);
        v[1] = norm2(rn0) + norm2(rn1);
        v[2] = dot_re(rn0, sn0) + dot_re(rn1, sn1);
        v[3] = norm2(sn0) + norm2(sn1);
    }
    write_partials<4>(v, Qc, g.nlog, w.logical);
}

void launch_cg_iter(const Geo &g, const CGIterFields &f, bool mixed, int slot, double tol,
                    bool decide_only, int sample, size_t lds_bytes, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1) {
    if (mixed)
        launch_stamped(k_cg_iter<true>, dim3(g.nblocks), dim3(g.block), lds_bytes, s, ev0, ev1, g, f,
                       slot, tol * tol, decide_only ? 1 : 0, sample);
    else
        launch_stamped(k_cg_iter<false>, dim3(g.nblocks), dim3(g.block), lds_bytes, s, ev0, ev1, g, f,
                       slot, tol * tol, decide_only ? 1 : 0, sample);
}

// The dynamic LDS granted so far to a kernel on each device (the attribute is set on the
// current device); 64 KiB is available without opting in.
struct LdsGrant {
    std::map<int, size_t> granted;
    std::mutex mu;  // contexts may run on several host threads
    int raise(const void *fn, size_t lds) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) {
            (void)hipGetLastError();
            return -1;
        }
        std::lock_guard<std::mutex> lock(mu);
        auto it = granted.emplace(dev, (size_t)64 * 1024).first;
        if (lds <= it->second) return 0;
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
            (void)hipGetLastError();  // clear the error state: the caller falls back
            return -1;
        }
        it->second = lds;
        return 0;
    }
};

int grant_cg_iter_lds(size_t lds_bytes) {
    static LdsGrant grant[2];
    if (grant[0].raise((const void *)k_cg_iter<false>, lds_bytes)) return -1;
    return grant[1].raise((const void *)k_cg_iter<true>, lds_bytes);
}

// ---------------------------------------------------------------- persistent small-chain CG
// One workgroup runs a whole solve for one small chain.  The search direction p and
// t = D p live in LDS (dynamic shared memory, 2 x 2V complex); r, x, the site geometry and
// the chain's links live in registers; the reductions are workgroup-local.  Mixed precision
// recomputes the residual in FP64 through global memory (x64, t64, r32) whenever the FP32
// residual has dropped by delta, exactly as the slot kernels do; that rare step is kept out
// of line so that its FP64 operands do not occupy registers in the iteration loop.  Each
// thread owns the chain-local sites tid + k * blockDim, k < SPT.  The final state is
// written to both state parities.

// t64 = D x64 on this thread's sites.
__device__ __noinline__ void wg_dx64(ChainInfo ci, CGFields f, int Vtot, int spt) {
    for (int k = 0; k < spt; ++k) {
        const int local = threadIdx.x + k * blockDim.x;
        if (local >= ci.V) break;
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int q, double2 &b0, double2 &b1) { b0 = f.x64[q]; b1 = f.x64[(size_t)Vtot + q]; };
        double2 o0, o1;
        dslash_site<double, false>(nb, s.flat, Vtot, f.U64, f.x64[s.flat],
                                   f.x64[(size_t)Vtot + s.flat], 2.0 + ci.m0, load, o0, o1);
        f.t64[s.flat] = o0;
        f.t64[(size_t)Vtot + s.flat] = o1;
    }
}

// r = phi - D^dagger t64 on this thread's sites, stored as r32; returns the local ||r||^2.
__device__ __noinline__ double wg_res64(ChainInfo ci, CGFields f, int Vtot, int spt) {
    double acc = 0.0;
    for (int k = 0; k < spt; ++k) {
        const int local = threadIdx.x + k * blockDim.x;
        if (local >= ci.V) break;
        const Site s = decode_site(ci, local);
        const Nbr nb = neighbours(ci, s);
        auto load = [&](int q, double2 &b0, double2 &b1) { b0 = f.t64[q]; b1 = f.t64[(size_t)Vtot + q]; };
        double2 a0, a1;
        dslash_site<double, true>(nb, s.flat, Vtot, f.U64, f.t64[s.flat],
                                  f.t64[(size_t)Vtot + s.flat], 2.0 + ci.m0, load, a0, a1);
        double2 h0, h1;
        sp_load(f.phi, Vtot, s.flat, h0, h1);
        const double2 r0 = make_double2(h0.x - a0.x, h0.y - a0.y);
        const double2 r1 = make_double2(h1.x - a1.x, h1.y - a1.y);
        sp_store(f.r32, Vtot, s.flat, make_float2((float)r0.x, (float)r0.y),
                 make_float2((float)r1.x, (float)r1.y));
        acc += norm2(r0) + norm2(r1);
    }
    return acc;
}

template <bool MIXED, int SPT>
__global__ void __launch_bounds__(1024)
k_cg_wg(Geo g, CGFields f, const int *__restrict__ chain_list, double tol2, double delta2,
        int max_iter) {
    using R = typename Prec<MIXED>::R;
    using C = cplx_t<R>;
    const int c = chain_list[blockIdx.x];
    const ChainInfo ci = g.chains[c];
    const int V = ci.V, Vtot = g.Vtot, off = ci.off;
    C *ps = (C *)smem_d;  // [2][V]
    C *ts = ps + 2 * V;   // [2][V]
    const LinkSrc<MIXED> U = link_source<MIXED>(f);
    const R mass = (R)(2.0 + ci.m0);

    Nbr nb[SPT];
    int fl[SPT];
    bool ok[SPT];
    C r[SPT][2], x[SPT][2], p[SPT][2];
    double v[1] = {0.0};
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int local = threadIdx.x + k * blockDim.x;
        ok[k] = local < V;
        fl[k] = off + (ok[k] ? local : 0);
        const Site s = decode_site(ci, ok[k] ? local : 0);
        nb[k] = neighbours(ci, s);
        for (int sp = 0; sp < 2; ++sp) {
            const double2 a = ok[k] ? f.phi[(size_t)sp * Vtot + fl[k]] : make_double2(0.0, 0.0);
            r[k][sp] = cmake<C>((R)a.x, (R)a.y);
            x[k][sp] = cmake<C>((R)0, (R)0);
            p[k][sp] = r[k][sp];
            v[0] += norm2(a);
            if (ok[k]) {
                if (MIXED) f.x64[(size_t)sp * Vtot + fl[k]] = make_double2(0.0, 0.0);
                ps[sp * V + (fl[k] - off)] = p[k][sp];
            }
        }
    }
    block_sum_all<1>(v);  // also makes ps visible
    const double phi2 = v[0], target = tol2 * v[0];
    double rho = v[0], rho_prev = v[0], rmax2 = v[0];
    int iters = 0, nupd = 0;
    bool conv = rho <= target;
    bool finite = isfinite(rho);
    auto loadP = [&](int q, C &b0, C &b1) { b0 = ps[q - off]; b1 = ps[V + q - off]; };
    auto loadT = [&](int q, C &b0, C &b1) { b0 = ts[q - off]; b1 = ts[V + q - off]; };
    while (!conv && finite && iters < max_iter) {
        // t = D p
        v[0] = 0.0;
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            if (!ok[k]) continue;
            C o0, o1;
            dslash_site<R, false>(nb[k], fl[k], Vtot, U, p[k][0], p[k][1], mass, loadP, o0, o1);
            ts[fl[k] - off] = o0;
            ts[V + fl[k] - off] = o1;
            v[0] += norm2(o0) + norm2(o1);
        }
        v[0] = block_sum_bcast(v[0], 0);  // also makes ts visible
        const R alpha = (R)(rho / v[0]);
        // x += alpha p, r -= alpha D^dagger t
        v[0] = 0.0;
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            if (!ok[k]) continue;
            C a0, a1;
            dslash_site<R, true>(nb[k], fl[k], Vtot, U, ts[fl[k] - off], ts[V + fl[k] - off], mass,
                                 loadT, a0, a1);
            const C Ap[2] = {a0, a1};
            for (int sp = 0; sp < 2; ++sp) {
                x[k][sp].x += alpha * p[k][sp].x; x[k][sp].y += alpha * p[k][sp].y;
                r[k][sp].x -= alpha * Ap[sp].x; r[k][sp].y -= alpha * Ap[sp].y;
                v[0] += norm2(r[k][sp]);
            }
        }
        v[0] = block_sum_bcast(v[0], 1);
        const double rho_new = v[0];
        ++iters;
        double beta = rho_new / rho;
        rho_prev = rho;
        rho = rho_new;
        if (!isfinite(rho_new)) { finite = false; break; }
        if (!MIXED) {
            if (rho_new <= target) { conv = true; break; }
        } else if (rho_new <= target || rho_new <= delta2 * rmax2) {
            // FP64 residual recomputation: x64 += x32; t64 = D x64; r = phi - D^dagger t64.
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                if (!ok[k]) continue;
                for (int sp = 0; sp < 2; ++sp) {
                    const size_t q = (size_t)sp * Vtot + fl[k];
                    const double2 xx = f.x64[q];
                    f.x64[q] = make_double2(xx.x + (double)x[k][sp].x, xx.y + (double)x[k][sp].y);
                    x[k][sp] = cmake<C>((R)0, (R)0);
                }
            }
            __syncthreads();
            wg_dx64(ci, f, Vtot, SPT);
            __syncthreads();
            v[0] = wg_res64(ci, f, Vtot, SPT);
            block_sum_all<1>(v);
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                if (!ok[k]) continue;
                const float4 rr = f.r32[fl[k]];
                r[k][0] = cmake<C>((R)rr.x, (R)rr.y);
                r[k][1] = cmake<C>((R)rr.z, (R)rr.w);
            }
            ++nupd;
            rmax2 = v[0];
            if (v[0] <= target) { rho = v[0]; conv = true; break; }
            if (!isfinite(v[0])) { rho = v[0]; finite = false; break; }
            beta = v[0] / rho_prev;
            rho = v[0];
        }
        // p = r + beta p
        const R b = (R)beta;
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            if (!ok[k]) continue;
            for (int sp = 0; sp < 2; ++sp) {
                p[k][sp].x = r[k][sp].x + b * p[k][sp].x;
                p[k][sp].y = r[k][sp].y + b * p[k][sp].y;
                ps[sp * V + (fl[k] - off)] = p[k][sp];
            }
        }
        __syncthreads();
    }
    // solution out
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        if (!ok[k]) continue;
        for (int sp = 0; sp < 2; ++sp) {
            const size_t q = (size_t)sp * Vtot + fl[k];
            if (MIXED) {
                const double2 xx = f.x64[q];
                f.x64[q] = make_double2(xx.x + (double)x[k][sp].x, xx.y + (double)x[k][sp].y);
            } else {
                f.x64[q] = make_double2((double)x[k][sp].x, (double)x[k][sp].y);
            }
        }
    }
    if (threadIdx.x == 0) {
        for (int par = 0; par < 2; ++par) {
            CGState *o = f.st + (size_t)par * g.nchains + c;
            o->rho = rho; o->rho_p = rho_prev; o->target = target; o->phi2 = phi2; o->rmax2 = rmax2;
            o->beta = 0.0; o->delta2 = delta2; o->alpha = 0.0; o->iters = iters;
            o->converged = conv ? kConverged : !finite ? kStopNonFinite : kStopMaxIter;
            o->mode = kModeNormal; o->n_updates = nupd;
        }
    }
}

// Dynamic LDS above 64 KiB must be opted in per kernel; the grant is remembered per
// instantiation and device.  Returns -1 (error state cleared) if the device refuses.
template <bool MIXED, int SPT> static int grant_wg_lds(size_t lds) {
    static LdsGrant grant;
    return grant.raise((const void *)k_cg_wg<MIXED, SPT>, lds);
}

template <bool MIXED, int SPT>
static int launch_wg_inst(const Geo &g, const CGFields &f, const int *chains, int n, int block,
                          double tol, double delta, int max_iter, size_t lds, hipStream_t s) {
    if (grant_wg_lds<MIXED, SPT>(lds)) return -1;
    hipLaunchKernelGGL((k_cg_wg<MIXED, SPT>), dim3(n), dim3(block), lds, s, g, f, chains, tol * tol,
                       delta * delta, max_iter);
    return 0;
}

int prepare_cg_wg(int vmax, bool mixed) {
    const size_t lds = cg_wg_lds_bytes(vmax, mixed);
    const int spt = vmax > 1024 ? 2 : 1;
    if (vmax > 2048) return -1;
    if (mixed) return spt == 1 ? grant_wg_lds<true, 1>(lds) : grant_wg_lds<true, 2>(lds);
    return spt == 1 ? grant_wg_lds<false, 1>(lds) : grant_wg_lds<false, 2>(lds);
}

size_t cg_wg_lds_bytes(int vmax, bool mixed) {
    return (size_t)4 * vmax * (mixed ? sizeof(float2) : sizeof(double2));
}

int launch_cg_wg(const Geo &g, const CGFields &f, bool mixed, const int *chains, int n, int vmax,
                 double tol, double delta, int max_iter, hipStream_t s) {
    if (n <= 0) return 0;
    const size_t lds = cg_wg_lds_bytes(vmax, mixed);
    // threads: the chain's sites over at most 4 per thread, in whole wavefronts
    int spt = 1;
    while ((vmax + spt - 1) / spt > 1024) spt *= 2;
    if (spt > 2) return -1;
    int block = (vmax + spt - 1) / spt;
    block = (block + 63) / 64 * 64;
    if (mixed) {
        if (spt == 1) return launch_wg_inst<true, 1>(g, f, chains, n, block, tol, delta, max_iter, lds, s);
        return launch_wg_inst<true, 2>(g, f, chains, n, block, tol, delta, max_iter, lds, s);
    }
    if (spt == 1) return launch_wg_inst<false, 1>(g, f, chains, n, block, tol, delta, max_iter, lds, s);
    return launch_wg_inst<false, 2>(g, f, chains, n, block, tol, delta, max_iter, lds, s);
}

// Order-preserving compaction of the workgroups of unconverged chains (one workgroup).
// A chain is dropped once either state parity says converged (a chain leaves the grid
// right after convergence, so its other parity may still hold the state before it).
// count[1] receives the number of unconverged chains that still have iterations left
// (iters < max_iter).
__global__ void __launch_bounds__(1024)
k_compact(const BlockWork *__restrict__ work, int n, CGState *__restrict__ st,
          const ChainInfo *__restrict__ chains, int nchains, int max_iter,
          BlockWork *__restrict__ out, int *count) {
    // The list is taken kEntries * blockDim.x entries at a time; thread t holds entries
    // t, t + B, t + 2B, ... of the round in registers.  All loads of a round are issued before
    // any of them is used, so a round costs two memory latencies, and one barrier orders it.
    constexpr int kEntries = 4;
    __shared__ int cnt[kEntries][kMaxWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int B = (int)blockDim.x;
    const unsigned long long below = (1ull << lane) - 1ull;
    int base = 0;
    double live[1] = {0.0};
    for (int r0 = 0; r0 < n; r0 += kEntries * B) {
        BlockWork wk[kEntries];
        bool valid[kEntries], keep[kEntries];
#pragma unroll
        for (int k = 0; k < kEntries; ++k) {
            const int i = r0 + k * B + (int)threadIdx.x;
            valid[k] = i < n;
            wk[k] = work[valid[k] ? i : 0];
        }
        int c0[kEntries], c1[kEntries], lead[kEntries], left[kEntries];
#pragma unroll
        for (int k = 0; k < kEntries; ++k) {
            const int c = wk[k].chain;
            c0[k] = st[c].converged;
            c1[k] = st[nchains + c].converged;
            lead[k] = wk[k].logical == chains[c].block0;
            left[k] = st[c].iters < max_iter || st[nchains + c].iters < max_iter;
        }
#pragma unroll
        for (int k = 0; k < kEntries; ++k) {
            keep[k] = valid[k] && !c0[k] && !c1[k];
            if (valid[k] && lead[k]) {  // once per chain
                if (keep[k] && left[k]) live[0] += 1.0;
                // A chain that converged in the last slot before this check is dropped with
                // only that slot's parity marked; the other parity still holds the state one
                // slot earlier.  Copying the final state over it keeps the chain's decision,
                // owed x update included, from being taken again by a later launch that reads
                // that parity.  (Either way at least one parity reads converged, so the keep
                // decisions of the chain's other entries do not depend on this copy.)
                const int c = wk[k].chain;
                if (c0[k] != c1[k]) {
                    if (c0[k]) st[nchains + c] = st[c];
                    else st[c] = st[nchains + c];
                }
            }
            const unsigned long long m = __ballot(keep[k]);
            if (lane == 0) cnt[k][wave] = __popcll(m);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kEntries; ++k) {
            int off = base, tot = 0;
            for (int v = 0; v < nw; ++v) {
                const int x = cnt[k][v];
                off += v < wave ? x : 0;
                tot += x;
            }
            const unsigned long long m = __ballot(keep[k]);
            if (keep[k]) out[off + __popcll(m & below)] = wk[k];
            base += tot;
        }
        __syncthreads();  // cnt is rewritten by the next round
    }
    block_sum_all<1>(live);
    if (threadIdx.x == 0) {
        count[0] = base;
        count[1] = (int)live[0];
    }
}

void launch_compact(const Geo &full, CGState *st, int max_iter, BlockWork *out, int *count,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, full.work, full.nblocks, st,
                       full.chains, full.nchains, max_iter, out, count);
}

__global__ void k_count_converged(const CGState *__restrict__ st, int n, int *out) {
    double v[1] = {0.0};
    for (int c = threadIdx.x; c < n; c += blockDim.x) v[0] += st[c].converged == kConverged;
    block_sum_all<1>(v);
    if (threadIdx.x == 0) out[0] = (int)v[0];
}

void launch_count_converged(const CGState *st_par, int n, int *out, hipStream_t s) {
    hipLaunchKernelGGL(k_count_converged, dim3(1), dim3(256), 0, s, st_par, n, out);
}

// ||phi - D^dagger t||^2 per chain, t = D x computed before.
__global__ void k_residual64(Geo g, const double2 *__restrict__ U, const double2 *__restrict__ phi,
                             const double2 *__restrict__ t, double *partials) {
    double v[1] = {0.0};
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    const Nbr nb = neighbours(ci, s);
    auto load = [&](int fl, double2 &b0, double2 &b1) { b0 = t[fl]; b1 = t[(size_t)Vtot + fl]; };
    double2 a0, a1;
    dslash_site<double, true>(nb, s.flat, Vtot, U, t[s.flat], t[(size_t)Vtot + s.flat],
                              2.0 + ci.m0, load, a0, a1);
    const double2 ph0 = phi[s.flat], ph1 = phi[(size_t)Vtot + s.flat];
    v[0] += norm2(make_double2(ph0.x - a0.x, ph0.y - a0.y)) +
            norm2(make_double2(ph1.x - a1.x, ph1.y - a1.y));
    SITES_END
    write_partials<1>(v, partials, g.nlog, w.logical);
}

void launch_true_residual64(const Geo &g, const double2 *U, const double2 *phi, const double2 *x,
                            double2 *t, double *partials, double *out, hipStream_t s) {
    launch_dslash64(g, U, x, t, false, s);
    hipLaunchKernelGGL(k_residual64, dim3(g.nblocks), dim3(g.block), 0, s, g, U, phi, t, partials);
    launch_finalize<1>(g, partials, out, s);
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
    SITES_BEGIN
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
    SITES_END
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
// Each thread takes sin theta of its own sites' plaquettes and stages them in LDS; the
// neighbours' plaquettes (n - x, n - t) come from there when the workgroup owns them and are
// recomputed (the same operations) otherwise.  KICK: p += c (F + add) instead of F = F + add.
template <bool KICK>
__global__ void k_gauge_force(Geo g, const double *__restrict__ q, const double *add, double c,
                              double *F) {
    double *sin_lds = smem_d;
    const BlockWork w = g.work[blockIdx.x];
    const ChainInfo ci = g.chains[w.chain];
    const int Vtot = g.Vtot;
    const int half = (int)blockDim.x >> 1;
    const int span = half * w.spt;
    const int par = (int)threadIdx.x >= half ? 1 : 0;
    for (int j = 0; j < w.spt; ++j) {
        const int i = w.start + (int)threadIdx.x - par * half + j * half;
        if (i >= ci.Vh) break;
        const Site s = decode_site(ci, par * ci.Vh + i);
        sin_lds[par * span + i - w.start] = sin(plaq_angle(ci, q, Vtot, s.x, s.t));
    }
    __syncthreads();
    auto sin_at = [&](int x, int t) {
        const int k = lds_slot(ci, w, span, flat_of(ci, x, t));
        return k >= 0 ? sin_lds[k] : sin(plaq_angle(ci, q, Vtot, x, t));
    };
    for (int j = 0; j < w.spt; ++j) {
        const int i = w.start + (int)threadIdx.x - par * half + j * half;
        if (i >= ci.Vh) break;
        const Site s = decode_site(ci, par * ci.Vh + i);
        const double sn = sin_lds[par * span + i - w.start];
        double fx = ci.beta * (sn - sin_at(s.x, wrap_dec(s.t, ci.Lt)));
        double ft = ci.beta * (sin_at(wrap_dec(s.x, ci.Lx), s.t) - sn);
        if (add) {
            fx += add[s.flat];
            ft += add[(size_t)Vtot + s.flat];
        }
        if (KICK) {
            F[s.flat] = F[s.flat] + c * fx;
            F[(size_t)Vtot + s.flat] = F[(size_t)Vtot + s.flat] + c * ft;
        } else {
            F[s.flat] = fx;
            F[(size_t)Vtot + s.flat] = ft;
        }
    }
}

void launch_gauge_force(const Geo &g, const double *q, const double *add, double *F, hipStream_t s) {
    hipLaunchKernelGGL(k_gauge_force<false>, dim3(g.nblocks), dim3(g.block), (size_t)2 * g.block * sizeof(double),
                       s, g, q, add, 0.0, F);
}

void launch_gauge_kick(const Geo &g, const double *q, const double *add, double c, double *p,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_gauge_force<true>, dim3(g.nblocks), dim3(g.block), (size_t)2 * g.block * sizeof(double),
                       s, g, q, add, c, p);
}

// ================================================================ Hessian-vector products
// The derivative of D along a link-field direction v, dD[v] = sum_a v_a dD/dq_a, is the
// hopping part of D with every fermion link U_mu(n) replaced by i v_mu(n) U_mu(n), since each
// link enters D as exp(i q).  k_weight_links writes those weighted links.
__global__ void k_weight_links(Geo g, const double2 *__restrict__ U, const double *__restrict__ v,
                               double2 *__restrict__ W) {
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    for (int mu = 0; mu < 2; ++mu) {
        const size_t l = (size_t)mu * Vtot + s.flat;
        W[l] = cscale(cmuli(U[l]), v[l]);
    }
    SITES_END
}

void launch_weight_links(const Geo &g, const double2 *U, const double *v, double2 *W,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_weight_links, dim3(g.nblocks), dim3(g.block), 0, s, g, U, v, W);
}

// out = S(L1; in1) [+ H(L2; in2)] [- sub], where S is the Wilson stencil with links L1 and mass
// term 2 + m0 (mass1 != 0) or its hopping part alone (mass1 == 0), and H the hopping part
// with links L2; DAG applies the dagger form to every stencil.
template <bool DAG>
__global__ void k_stencil2(Geo g, const double2 *__restrict__ L1, const double2 *__restrict__ in1,
                           int mass1, const double2 *__restrict__ L2,
                           const double2 *__restrict__ in2, const double2 *__restrict__ sub,
                           double2 *__restrict__ out) {
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    const Nbr nb = neighbours(ci, s);
    auto load1 = [&](int f, double2 &b0, double2 &b1) { b0 = in1[f]; b1 = in1[(size_t)Vtot + f]; };
    double2 o0, o1;
    dslash_site<double, DAG>(nb, s.flat, Vtot, L1, in1[s.flat], in1[(size_t)Vtot + s.flat],
                             mass1 ? 2.0 + ci.m0 : 0.0, load1, o0, o1);
    if (in2) {
        auto load2 = [&](int f, double2 &b0, double2 &b1) { b0 = in2[f]; b1 = in2[(size_t)Vtot + f]; };
        double2 h0, h1;
        const double2 zero = make_double2(0.0, 0.0);
        dslash_site<double, DAG>(nb, s.flat, Vtot, L2, zero, zero, 0.0, load2, h0, h1);
        o0 = cadd(o0, h0);
        o1 = cadd(o1, h1);
    }
    if (sub) {
        o0 = csub(o0, sub[s.flat]);
        o1 = csub(o1, sub[(size_t)Vtot + s.flat]);
    }
    out[s.flat] = o0;
    out[(size_t)Vtot + s.flat] = o1;
    SITES_END
}

void launch_stencil2(const Geo &g, bool dagger, const double2 *L1, const double2 *in1, bool mass1,
                     const double2 *L2, const double2 *in2, const double2 *sub, double2 *out,
                     hipStream_t s) {
    if (dagger)
        hipLaunchKernelGGL(k_stencil2<true>, dim3(g.nblocks), dim3(g.block), 0, s, g, L1, in1,
                           mass1 ? 1 : 0, L2, in2, sub, out);
    else
        hipLaunchKernelGGL(k_stencil2<false>, dim3(g.nblocks), dim3(g.block), 0, s, g, L1, in1,
                           mass1 ? 1 : 0, L2, in2, sub, out);
}

// The two hopping bilinears of the link (n, mu) for spinor fields X, Y:
//   T1 = X(n)^dagger (1 - sigma_mu) U_mu(n) Y(n + mu),
//   T2 = X(n + mu)^dagger (1 + sigma_mu) U_mu^dagger(n) Y(n),
// through the rank-one projector forms of the force kernel.
struct LinkSpinors {
    double2 a0, a1;  // field at n
    double2 b0, b1;  // field at n + mu
};
__device__ __forceinline__ LinkSpinors link_spinors(const double2 *__restrict__ f, int Vtot, int n,
                                                    int nmu) {
    LinkSpinors r;
    r.a0 = f[n]; r.a1 = f[(size_t)Vtot + n];
    r.b0 = f[nmu]; r.b1 = f[(size_t)Vtot + nmu];
    return r;
}
template <int MU>
__device__ __forceinline__ void bilinears(const LinkSpinors &X, const LinkSpinors &Y, double2 u,
                                          double2 &T1, double2 &T2) {
    if (MU == 0) {
        T1 = cmulc(csub(X.a0, X.a1), cmul(u, csub(Y.b0, Y.b1)));
        T2 = cmulc(cadd(X.b0, X.b1), cmulc(u, cadd(Y.a0, Y.a1)));
    } else {
        T1 = cmulc(cadd(X.a0, cmuli(X.a1)), cmul(u, cadd(Y.b0, cmuli(Y.b1))));
        T2 = cmulc(csub(X.b0, cmuli(X.b1)), cmulc(u, csub(Y.a0, cmuli(Y.a1))));
    }
}

// (H v)_a for S_F = phi^dagger (D^dagger D)^{-1} phi at the link a = (n, mu).  With
// xi = (D^dagger D)^{-1} phi, chi = D xi, dD_a = dD/dq_a:
//   (H v)_a = 2 Re[ Z1^dagger dD_a xi + chi^dagger dD_a Z2 - v_a chi^dagger d2D_a xi ],
//   Z2 = D^{-1} (dD[v] xi + Z1), Z1 = D^{dagger -1} dD[v]^dagger chi   (Sec. 3, Eqs. (21)-(23)).
// Here Z2 = (D^dagger D)^{-1} (D^dagger dD[v] xi + dD[v]^dagger chi), one normal-equation
// solve, and Z1 = D Z2 - dD[v] xi.  dD_a has the entries -(i/2)(1 - sigma_mu) U at
// (n, n+mu) and (i/2)(1 + sigma_mu) U^dagger at (n+mu, n); d2D_a is minus the hopping entries,
// so with T1, T2 above:
//   2 Re[X^dagger dD_a Y] = Im(T1 - T2),   2 Re[X^dagger d2D_a Y] = Re(T1 + T2).
template <int MU>
__device__ __forceinline__ double hvp_fermion_link(const LinkSpinors &chi, const LinkSpinors &xi,
                                                   const LinkSpinors &z1, const LinkSpinors &z2,
                                                   double2 u, double va) {
    double2 t1, t2, s1, s2, c1, c2;
    bilinears<MU>(z1, xi, u, t1, t2);
    bilinears<MU>(chi, z2, u, s1, s2);
    bilinears<MU>(chi, xi, u, c1, c2);
    return (t1.y - t2.y) + (s1.y - s2.y) - va * (c1.x + c2.x);
}

// out = scale * (H v) for the action selected by the pointers: the fermion part when chi is
// given (xi, z1, z2 as above), the gauge part when gauge != 0.  The gauge part follows from
// F_x(n) = beta [sin th(n) - sin th(n - t)], F_t(n) = beta [sin th(n - x) - sin th(n)]:
//   (H_G v)_x(n) = beta [cos th(n) dth(n) - cos th(n - t) dth(n - t)],
//   (H_G v)_t(n) = beta [cos th(n - x) dth(n - x) - cos th(n) dth(n)],
// with dth the plaquette combination of v.
__global__ void k_hessian_vector(Geo g, const double2 *__restrict__ U, const double *__restrict__ v,
                                 const double2 *__restrict__ chi, const double2 *__restrict__ xi,
                                 const double2 *__restrict__ z1, const double2 *__restrict__ z2,
                                 const double *__restrict__ q, int gauge, double scale,
                                 double *__restrict__ out) {
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    const size_t lx = s.flat, lt = (size_t)Vtot + s.flat;
    double hx = 0.0, ht = 0.0;
    if (chi) {
        const int nxp = flat_of(ci, wrap_inc(s.x, ci.Lx), s.t);
        const int ntp = flat_of(ci, s.x, wrap_inc(s.t, ci.Lt));
        {
            const LinkSpinors C = link_spinors(chi, Vtot, s.flat, nxp), X = link_spinors(xi, Vtot, s.flat, nxp);
            const LinkSpinors A = link_spinors(z1, Vtot, s.flat, nxp), B = link_spinors(z2, Vtot, s.flat, nxp);
            hx += hvp_fermion_link<0>(C, X, A, B, U[lx], v[lx]);
        }
        {
            const LinkSpinors C = link_spinors(chi, Vtot, s.flat, ntp), X = link_spinors(xi, Vtot, s.flat, ntp);
            const LinkSpinors A = link_spinors(z1, Vtot, s.flat, ntp), B = link_spinors(z2, Vtot, s.flat, ntp);
            ht += hvp_fermion_link<1>(C, X, A, B, U[lt], v[lt]);
        }
    }
    if (gauge) {
        const int tm = wrap_dec(s.t, ci.Lt), xm = wrap_dec(s.x, ci.Lx);
        const double a0 = cos(plaq_angle(ci, q, Vtot, s.x, s.t)) * plaq_angle(ci, v, Vtot, s.x, s.t);
        const double at = cos(plaq_angle(ci, q, Vtot, s.x, tm)) * plaq_angle(ci, v, Vtot, s.x, tm);
        const double ax = cos(plaq_angle(ci, q, Vtot, xm, s.t)) * plaq_angle(ci, v, Vtot, xm, s.t);
        hx += ci.beta * (a0 - at);
        ht += ci.beta * (ax - a0);
    }
    out[lx] = scale * hx;
    out[lt] = scale * ht;
    SITES_END
}

void launch_hessian_vector(const Geo &g, const double2 *U, const double *v, const double2 *chi,
                           const double2 *xi, const double2 *z1, const double2 *z2,
                           const double *q, bool gauge, double scale, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_hessian_vector, dim3(g.nblocks), dim3(g.block), 0, s, g, U, v, chi, xi,
                       z1, z2, q, gauge ? 1 : 0, scale, out);
}

// ================================================================ updates
// blockIdx.y selects the plane (mu); the sites [site0, site0 + n) of both planes
__global__ void k_axpy(const double *__restrict__ a, double c, const double *__restrict__ b,
                       double *__restrict__ out, size_t site0, size_t n, size_t plane) {
    const size_t base = blockIdx.y * plane + site0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[base + i] = a[base + i] + c * b[base + i];
}

void launch_axpy_links(const Geo &g, const double *a, double c, const double *b, double *out,
                       hipStream_t s) {
    const size_t n = (size_t)g.nsites;
    const int block = 256;
    size_t grid = (n + block - 1) / block;
    if (grid > 32768) grid = 32768;
    if (n == 0) return;
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)grid, 2), dim3(block), 0, s, a, c, b, out,
                       (size_t)g.site0, n, (size_t)g.Vtot);
}

void launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    (void)hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

// ================================================================ random numbers
// Box-Muller pair from Philox words: r = sqrt(-2 ln(1 - ua)), (r cos 2 pi ub, r sin 2 pi ub),
// with ln, sin and cos taken by one written method (Cody and Waite's argument reduction, then
// truncated series with exact reciprocal coefficients), evaluated with IEEE operations only
// (+, -, *, / and sqrt rounded to nearest, no contraction into fused multiply-adds), so the
// momenta and pseudofermions of Sec. 2.1 have the same bits on any host that evaluates the
// same operations in the same order.

// ln y for 0 < y <= 1: y = m 2^e with m in [1/sqrt 2, sqrt 2); with f = (m-1)/(m+1) and
// s = f^2, ln m = 2 atanh f = 2 (f + f s A(s)), A(s) = sum_{k=1..11} s^(k-1) / (2k+1)
// (|f| <= 0.1716); ln y = (e C2 + ln m) + e C1, where C1 = 355/512 is exact in 9 bits
// and C2 = ln 2 - C1 (rounded).
__device__ __forceinline__ double bm_log(double y) {
#pragma clang fp contract(off)
    int e = 0;
    double m = frexp(y, &e);
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e -= 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double s = f * f;
    double a = 1.0 / 23.0;
#pragma unroll
    for (int k = 21; k >= 3; k -= 2) a = 1.0 / (double)k + s * a;
    const double lnm = 2.0 * (f + f * (s * a));
    const double de = (double)e;
    return (de * -2.121944400546905827679e-4 + lnm) + de * 0.693359375;
}

// (sin 2 pi u, cos 2 pi u) for u in [0, 1), u a multiple of 2^-53.  The quadrant
// n = floor(4u + 1/2) and the offset d = u - n/4 in [-1/8, 1/8] are exact; x = 2 pi d is
// formed with 2 pi split into its rounded value and the rounded remainder; on |x| <= pi/4
// sin x = x - x (z S(z)), cos x = 1 - z K(z) with z = x^2 and the alternating series
// S = 1/3! - z/5! + ... - z^9/21!, K = 1/2! - z/4! + ... + z^10/22!, summed from the
// highest power down.
__device__ __forceinline__ void bm_sincos_turn(double u, double &sn, double &cs) {
#pragma clang fp contract(off)
    const double n = floor(4.0 * u + 0.5);
    const double d = u - 0.25 * n;
    const double x = d * 6.283185307179586 + d * 2.4492935982947064e-16;
    const double z = x * x;
    // 1/k! for k = 2..22 (each k! is exact in binary64 up to 22!)
    double fact[23];
    fact[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= 22; ++k) fact[k] = fact[k - 1] * (double)k;
    double S = -1.0 / fact[21];
#pragma unroll
    for (int k = 19; k >= 3; k -= 2) S = ((k & 2) ? 1.0 : -1.0) / fact[k] + z * S;
    double K = 1.0 / fact[22];
#pragma unroll
    for (int k = 20; k >= 2; k -= 2) K = ((k & 2) ? 1.0 : -1.0) / fact[k] + z * K;
    const double sx = x - x * (z * S);
    const double cx = 1.0 - z * K;
    switch ((int)n & 3) {
    case 0: sn = sx; cs = cx; break;
    case 1: sn = cx; cs = -sx; break;
    case 2: sn = -sx; cs = -cx; break;
    default: sn = -cx; cs = sx; break;
    }
}

__device__ __forceinline__ void gaussian_pair(const U32x4 &w, double &g0, double &g1) {
#pragma clang fp contract(off)
    const double ua = u01_from(w.v[0], w.v[1]), ub = u01_from(w.v[2], w.v[3]);
    const double r = __builtin_sqrt(-2.0 * bm_log(1.0 - ua));
    double sn, cs;
    bm_sincos_turn(ub, sn, cs);
    g0 = r * cs;
    g1 = r * sn;
}

__global__ void k_rng_links(Geo g, uint32_t k0, uint32_t k1, double *__restrict__ q) {
#pragma clang fp contract(off)
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    const uint32_t n = (uint32_t)(s.x + ci.Lx * s.t);
    for (int mu = 0; mu < 2; ++mu) {
        const U32x4 r = philox4x32_10(2 * n + mu, kStreamLinks, 0u, ci.chain_id, k0, k1);
        const double u = u01_from(r.v[0], r.v[1]);
        q[(size_t)mu * Vtot + s.flat] = 3.141592653589793 * (2.0 * u - 1.0);
    }
    SITES_END
}

void launch_rng_links(const Geo &g, uint64_t seed, double *q, hipStream_t s) {
    hipLaunchKernelGGL(k_rng_links, dim3(g.nblocks), dim3(g.block), 0, s, g, (uint32_t)seed,
                       (uint32_t)(seed >> 32), q);
}

__global__ void k_refresh(Geo g, uint32_t k0, uint32_t k1, const uint32_t *__restrict__ traj_dev,
                          double *__restrict__ p, double2 *__restrict__ zeta, int fermions,
                          double *partials) {
#pragma clang fp contract(off)
    const uint32_t traj = *traj_dev;
    double v[2] = {0.0, 0.0};
    SITES_BEGIN
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
    SITES_END
    write_partials<2>(v, partials, g.nlog, w.logical);
}

void launch_refresh(const Geo &g, uint64_t seed, const uint32_t *traj, double *p, double2 *zeta,
                    bool fermions, double *partials, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_refresh, dim3(g.nblocks), dim3(g.block), 0, s, g, (uint32_t)seed,
                       (uint32_t)(seed >> 32), traj, p, zeta, fermions ? 1 : 0, partials);
    launch_finalize<2>(g, partials, out, s);
}

// ================================================================ energies
__global__ void k_energy(Geo g, const double *__restrict__ q, const double *__restrict__ q0,
                         const double *__restrict__ p, const double *__restrict__ p0,
                         const double2 *__restrict__ phi, const double2 *__restrict__ xi,
                         double *partials) {
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    for (int mu = 0; mu < 2; ++mu) {
        const double a = p[(size_t)mu * Vtot + s.flat], b = p0[(size_t)mu * Vtot + s.flat];
        v[0] += 0.5 * (a - b) * (a + b);
        v[2] += 0.5 * a * a;
    }
    const double c1 = cos(plaq_angle(ci, q, Vtot, s.x, s.t));
    const double c0 = cos(plaq_angle(ci, q0, Vtot, s.x, s.t));
    v[1] += c0 - c1;
    v[3] += 1.0 - c1;
    v[4] += 1.0 - c0;
    v[6] += c1;
    if (phi) {
        for (int sp = 0; sp < 2; ++sp) {
            const double2 a = phi[(size_t)sp * Vtot + s.flat], b = xi[(size_t)sp * Vtot + s.flat];
            v[5] += a.x * b.x + a.y * b.y;
        }
    }
    SITES_END
    write_partials<7>(v, partials, g.nlog, w.logical);
}

void launch_energy(const Geo &g, const double *q, const double *q0, const double *p,
                   const double *p0, const double2 *phi, const double2 *xi, double *partials,
                   double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_energy, dim3(g.nblocks), dim3(g.block), 0, s, g, q, q0, p, p0, phi, xi,
                       partials);
    launch_finalize<7>(g, partials, out, s);
}

__global__ void k_gauge_energy(Geo g, const double *__restrict__ q, const double2 *__restrict__ phi,
                               const double2 *__restrict__ xi, double *partials) {
    double v[3] = {0, 0, 0};
    SITES_BEGIN
    const Site s = decode_site(ci, local);
    const double c1 = cos(plaq_angle(ci, q, Vtot, s.x, s.t));
    v[0] += 1.0 - c1;
    v[1] += c1;
    if (phi) {
        for (int sp = 0; sp < 2; ++sp) {
            const double2 a = phi[(size_t)sp * Vtot + s.flat], b = xi[(size_t)sp * Vtot + s.flat];
            v[2] += a.x * b.x + a.y * b.y;
        }
    }
    SITES_END
    write_partials<3>(v, partials, g.nlog, w.logical);
}

void launch_gauge_energy(const Geo &g, const double *q, const double2 *phi, const double2 *xi,
                         double *partials, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_gauge_energy, dim3(g.nblocks), dim3(g.block), 0, s, g, q, phi, xi, partials);
    launch_finalize<3>(g, partials, out, s);
}

// Delta H = sum 1/2 (p'^2 - p^2) + beta sum (cos theta - cos theta') + (S_F' - S_F), then
// accept iff Delta H <= 0 or u < exp(-Delta H) (Sec. 2.1).
__global__ void k_metropolis(Geo g, uint32_t k0, uint32_t k1, const uint32_t *__restrict__ traj_dev,
                             const double *__restrict__ es, const double *__restrict__ rs,
                             const int *__restrict__ cstat, MetroOut *out, int fermions) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nchains) return;
    const uint32_t traj = *traj_dev;
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

void launch_metropolis(const Geo &g, uint64_t seed, const uint32_t *traj, const double *esums,
                       const double *rsums, const int *chain_status, MetroOut *out, bool fermions,
                       hipStream_t s) {
    const int block = 64;
    hipLaunchKernelGGL(k_metropolis, dim3((g.nchains + block - 1) / block), dim3(block), 0, s, g,
                       (uint32_t)seed, (uint32_t)(seed >> 32), traj, esums, rsums, chain_status, out,
                       fermions ? 1 : 0);
}

__global__ void k_restore(Geo g, const MetroOut *__restrict__ m, const double *__restrict__ q0,
                          double *__restrict__ q) {
    SITES_BEGIN
    if (m[w.chain].accepted) break;
    const int fl = ci.off + local;
    q[fl] = q0[fl];
    q[(size_t)Vtot + fl] = q0[(size_t)Vtot + fl];
    SITES_END
}

// ================================================================ device-side bookkeeping
// Streaming copy, one 16-byte nontemporal load and store per thread: the measured
// bandwidth ceiling of the roofline figures and the calibration kernel of the HBM counters.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ void k_stream_copy(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

void launch_stream_copy(const void *src, void *dst, size_t n16, hipStream_t s) {
    const unsigned blocks = (unsigned)((n16 + 255) / 256);
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, s, (const f32x4 *)src,
                       (f32x4 *)dst, n16);
}

__global__ void k_iota(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

void launch_iota(int *p, int n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_iota, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

__global__ void k_set_u32(uint32_t *p, uint32_t v) { *p = v; }

void launch_set_u32(uint32_t *p, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, p, v);
}

// log[2c] = iterations, log[2c + 1] = stop code (CGState::converged) of chain c's finished solve
__global__ void k_log_solve(const CGState *__restrict__ st, int nchains, int *__restrict__ log) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchains) return;
    log[2 * c] = st[c].iters;
    log[2 * c + 1] = st[c].converged;
}

void launch_log_solve(const CGState *st, int nchains, int *log, hipStream_t s) {
    const int block = 256;
    hipLaunchKernelGGL(k_log_solve, dim3((nchains + block - 1) / block), dim3(block), 0, s, st,
                       nchains, log);
}

// status[c]: -3 (the library's "did not converge") or -5 (non-finite residual) from the first
// of the n logged solves of chain c that stopped unconverged, else 0
__global__ void k_chain_status(const int *__restrict__ log, int n, int nchains, int *__restrict__ status) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchains) return;
    int st = 0;
    for (int k = 0; k < n && st == 0; ++k) {
        const int code = log[((size_t)k * nchains + c) * 2 + 1];
        if (code != kConverged) st = code == kStopNonFinite ? -5 : -3;
    }
    status[c] = st;
}

void launch_chain_status(const int *log, int n, int nchains, int *status, hipStream_t s) {
    const int block = 256;
    hipLaunchKernelGGL(k_chain_status, dim3((nchains + block - 1) / block), dim3(block), 0, s, log, n,
                       nchains, status);
}

void launch_restore(const Geo &g, const MetroOut *m, const double *q0, double *q, hipStream_t s) {
    hipLaunchKernelGGL(k_restore, dim3(g.nblocks), dim3(g.block), 0, s, g, m, q0, q);
}

}  // namespace shmc
