// Internal types and device helpers of the Schwinger-model HMC library (gfx950).
//
// Lattice layout in device memory ("native" layout):
//   A batch holds C independent chains.  Chain c is an Lx_c x Lt_c lattice (both even)
//   with V_c = Lx_c * Lt_c sites.  All chains share one flat site space of
//   Vtot = sum_c V_c sites; chain c owns flat sites [off_c, off_c + V_c).
//   Inside a chain the sites are ordered even-odd (checkerboard): parity
//   par = (x + t) & 1 first, then i = t * (Lx/2) + x/2, so flat = off + par*Vh + i.
//   Consecutive threads touch consecutive i, so every stencil neighbour row is a
//   contiguous, coalesced stream.
//   Fields are structure-of-arrays over that flat space:
//     real link fields (angles q, momenta p, forces)  : [mu][Vtot]  double
//     complex links U_mu(n) = exp(i q_mu(n))          : [mu][Vtot]  double2 / float2
//     spinors (two complex components)                : [s][Vtot]   double2 / float2
//   mu = 0 is x (the paper's direction 1), mu = 1 is t (direction 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shmc {

constexpr int kMaxBlock = 1024;  // largest workgroup of the site kernels

struct ChainInfo {
    int off;      // first flat site
    int Lx, Lt;   // extents
    int hx;       // Lx / 2
    int Vh;       // V / 2
    int V;        // Lx * Lt
    int block0;   // first logical workgroup of this chain
    int nblocks;  // logical workgroups of this chain
    double beta;  // Wilson gauge coupling
    double m0;    // bare mass
    uint32_t chain_id;  // chain index used as the fourth Philox counter word
    int small;          // 1: its CG runs in the one-workgroup persistent solver
    int pad[2];
};
static_assert(sizeof(ChainInfo) == 64, "ChainInfo is 64 bytes");

// One entry per hardware workgroup (hardware order, XCD-aware permutation applied on the host).
// A workgroup of B threads handles the half-site indices [start, start + B/2) of BOTH parity
// planes of its chain: threads [0, B/2) the even plane, [B/2, B) the odd plane.  The stencil
// neighbours of a site lie in the other plane at nearby half-site indices, so the two halves
// of the workgroup read each other's sites while they are still in cache.
struct BlockWork {
    int chain;    // chain index
    int start;    // first half-site index (within each parity plane) of this workgroup
    int logical;  // logical workgroup index (chains are contiguous in logical order)
    int spt;      // sites per thread
};

struct Site {
    int local;  // chain-local site index in [0, V)
    int flat;   // flat index in [0, Vtot)
    int par;    // parity (x + t) & 1
    int x, t;
};

__device__ __forceinline__ Site decode_site(const ChainInfo &ci, int local) {
    Site s;
    s.local = local;
    s.flat = ci.off + local;
    s.par = local >= ci.Vh ? 1 : 0;
    int i = local - s.par * ci.Vh;
    s.t = i / ci.hx;
    int xh = i - s.t * ci.hx;
    s.x = 2 * xh + ((s.par ^ s.t) & 1);
    return s;
}

// flat index of the site (x, t) of chain ci (x, t already wrapped)
__device__ __forceinline__ int flat_of(const ChainInfo &ci, int x, int t) {
    int par = (x + t) & 1;
    return ci.off + par * ci.Vh + t * ci.hx + (x >> 1);
}

__device__ __forceinline__ int wrap_inc(int a, int L) { return a + 1 == L ? 0 : a + 1; }
__device__ __forceinline__ int wrap_dec(int a, int L) { return a == 0 ? L - 1 : a - 1; }

// ---------------------------------------------------------------- complex helpers
template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };
template <typename T> using cplx_t = typename Cplx<T>::type;

template <typename C> __device__ __forceinline__ C cmake(decltype(C::x) re, decltype(C::x) im) {
    C c; c.x = re; c.y = im; return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
    return cmake<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cmuli(C a) { return cmake<C>(-a.y, a.x); }   // i a
template <typename C> __device__ __forceinline__ C cmulmi(C a) { return cmake<C>(a.y, -a.x); }  // -i a
template <typename C, typename R> __device__ __forceinline__ C cscale(C a, R s) {
    return cmake<C>(a.x * s, a.y * s);
}

// ---------------------------------------------------------------- Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of two
// 32x32->64 multiplies, xor with the round key and the other counter words, and a word
// permutation; the key is bumped by the Weyl constants between rounds.
struct U32x4 { uint32_t v[4]; };

__device__ __forceinline__ U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    U32x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Random streams (counter word 1) and the counter convention
// (index, stream, trajectory, chain); key = (seed low, seed high).
enum Stream : uint32_t { kStreamLinks = 0, kStreamMomenta = 1, kStreamPseudofermion = 2, kStreamMetropolis = 3 };

__device__ __forceinline__ double u01_from(uint32_t lo, uint32_t hi) {
    uint64_t v = (uint64_t)lo | ((uint64_t)hi << 32);
    return (double)(v >> 11) * 0x1.0p-53;  // exact: 53-bit integer times a power of two
}

}  // namespace shmc
