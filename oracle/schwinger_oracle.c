/*
 * Plain FP64 CPU oracle for the HMC of the two-flavour lattice Schwinger model with
 * the (adapted) nested force-gradient integrators of Shcherbakov, Ehrhardt,
 * Finkenrath, Guenther, Knechtli and Peardon, "Adapted nested force-gradient
 * integrators: the Schwinger model case" (arXiv:1512.03812).
 *
 * THIS IS TEST INFRASTRUCTURE.  It exists only to check the GPU library.  Only the
 * test suite, the package smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the GPU path.  Everything is
 * written for clarity: plain loops, lexicographic layout, double precision,
 * `double complex`, no blocking, no fusion, no reordering beyond what the paper's
 * definitions state.
 *
 * Conventions
 *   lattice Lx x Lt, site n = x + Lx*t, direction mu = 0 is x (the paper's "1"),
 *   mu = 1 is t (the paper's "2").  Link angles q[2*n + mu]; U_mu(n) = exp(i q_mu(n))
 *   (Sec. 3).  Momenta p[2*n + mu] (real, the Lie algebra of U(1), Sec. 3).
 *   Spinors psi[2*n + s], s = 0, 1, complex (two-component, Sec. 3).
 *   Gauge field periodic in both directions.  Fermions periodic in x and
 *   antiperiodic in t: the sign is carried by the t-links leaving the last time
 *   slice (the paper does not state the boundary conditions; this is the reading
 *   used throughout).
 *
 * Parity pins for every function here live in the test suite (free-field spectrum,
 * adjointness and gamma5-hermiticity, gauge invariance, finite differences,
 * reversibility, order slopes, Philox known-answer vectors, exact quenched
 * plaquette, stage sequences typed from the paper's equations).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* Lattice geometry                                                          */
/* ------------------------------------------------------------------------- */

static int wrap(int a, int L) { return ((a % L) + L) % L; }

/* site index of (x, t) with periodic wrap */
static int site(int x, int t, int Lx, int Lt) { return wrap(x, Lx) + Lx * wrap(t, Lt); }

/* neighbour of n displaced by d (= +1 or -1) in direction mu */
static int hop(int n, int mu, int d, int Lx, int Lt)
{
    int x = n % Lx, t = n / Lx;
    if (mu == 0) x += d; else t += d;
    return site(x, t, Lx, Lt);
}

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers: Philox4x32-10                               */
/* Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", */
/* SC'11.  Round function: two 32x32->64 multiplies by the Philox            */
/* multipliers, a xor with the round key and the other counter words, and a   */
/* permutation; the key is bumped by the Weyl constants between rounds.       */
/* ------------------------------------------------------------------------- */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (round < 9) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * Stream definition shared (by specification, not by code) with the GPU path:
 *   key     = (seed low word, seed high word)
 *   counter = (index, stream, trajectory, chain)
 *   streams: 0 initial links, 1 momenta, 2 pseudofermion, 3 Metropolis
 *   index   : lexicographic link index 2n+mu (streams 0, 1), spinor index 2n+s
 *             (stream 2), 0 (stream 3)
 *   uniform : 64-bit word (w0 | w1 << 32) >> 11, times 2^-53, in [0, 1)
 *   gaussian pair (Box-Muller): r = sqrt(-2 ln(1 - ua)), (r cos(2 pi ub), r sin(2 pi ub)),
 *             with ln, sin and cos evaluated as below (orc_ln_unit, orc_sincos_turn)
 */
enum { STREAM_LINKS = 0, STREAM_MOMENTA = 1, STREAM_PSEUDOFERMION = 2, STREAM_METROPOLIS = 3 };

static void draw(uint64_t seed, uint32_t chain, uint32_t traj, uint32_t stream, uint32_t index,
                 uint32_t w[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {index, stream, traj, chain};
    orc_philox4x32_10(ctr, key, w);
}

static double u01(uint32_t lo, uint32_t hi)
{
    uint64_t v = (uint64_t)lo | ((uint64_t)hi << 32);
    return (double)(v >> 11) * 0x1.0p-53;
}

void orc_uniform_pair(uint64_t seed, uint32_t chain, uint32_t traj, uint32_t stream,
                      uint32_t index, double out[2])
{
    uint32_t w[4];
    draw(seed, chain, traj, stream, index, w);
    out[0] = u01(w[0], w[1]);
    out[1] = u01(w[2], w[3]);
}

/*
 * The logarithm and the sine and cosine of Box-Muller, written out so that the GPU path can
 * evaluate the same sequence of IEEE operations (+, -, *, / rounded to nearest; the file is
 * compiled without contraction into fused multiply-adds) and obtain the same bits.  The
 * method is the argument reduction of Cody and Waite (Software Manual for the Elementary
 * Functions, 1980) with truncated series whose coefficients are exact reciprocals:
 *
 * ln y, 0 < y <= 1:  y = m 2^e with m in [1/sqrt 2, sqrt 2) (frexp, exact);
 *   f = (m - 1) / (m + 1), s = f^2;  ln m = 2 atanh f = 2 (f + f s (1/3 + s (1/5 + ...
 *   + s (1/23)))) (|f| <= 0.1716, s <= 0.0295: the first omitted term is below 2^-60 of f);
 *   ln y = (e C2 + ln m) + e C1, with C1 = 355/512 and C2 = ln 2 - C1 rounded
 *   (C1 has 9 significant bits, so e C1 is exact).
 *
 * sin and cos of 2 pi u, 0 <= u < 1 (u a multiple of 2^-53):  n = floor(4u + 1/2) and
 *   d = u - n/4 in [-1/8, 1/8] (both exact); x = d P1 + d P2 with P1 + P2 = 2 pi
 *   (P1 = 2 pi rounded, P2 the rounded remainder), |x| <= pi/4;
 *   z = x^2, sin x = x - x (z Q), Q = 1/3! - z/5! + z^2/7! - ... - z^9/21!,
 *   cos x = 1 - z P, P = 1/2! - z/4! + z^2/6! - ... + z^10/22! (both by Horner's rule from
 *   the highest power; the first omitted terms are below 2^-60 of the result); the quadrant
 *   n mod 4 then rotates (sin x, cos x) by multiples of pi/2.
 */
double orc_ln_unit(double y)
{
    int e;
    double m = frexp(y, &e);                      /* y = m 2^e, m in [1/2, 1) */
    if (m < 0.70710678118654752440) { m = m * 2.0; e = e - 1; }
    const double f = (m - 1.0) / (m + 1.0);
    const double s = f * f;
    double poly = 1.0 / 23.0;
    poly = 1.0 / 21.0 + s * poly;
    poly = 1.0 / 19.0 + s * poly;
    poly = 1.0 / 17.0 + s * poly;
    poly = 1.0 / 15.0 + s * poly;
    poly = 1.0 / 13.0 + s * poly;
    poly = 1.0 / 11.0 + s * poly;
    poly = 1.0 / 9.0 + s * poly;
    poly = 1.0 / 7.0 + s * poly;
    poly = 1.0 / 5.0 + s * poly;
    poly = 1.0 / 3.0 + s * poly;
    const double lnm = 2.0 * (f + f * (s * poly));
    const double C1 = 0.693359375, C2 = -2.121944400546905827679e-4;
    const double de = (double)e;
    return (de * C2 + lnm) + de * C1;
}

void orc_sincos_turn(double u, double *sn, double *cs)
{
    const double n = floor(4.0 * u + 0.5);
    const double d = u - 0.25 * n;
    const double P1 = 6.283185307179586, P2 = 2.4492935982947064e-16;
    const double x = d * P1 + d * P2;
    const double z = x * x;
    double ps = -1.0 / 51090942171709440000.0;    /* -1/21! */
    ps = 1.0 / 121645100408832000.0 + z * ps;     /*  1/19! */
    ps = -1.0 / 355687428096000.0 + z * ps;       /* -1/17! */
    ps = 1.0 / 1307674368000.0 + z * ps;          /*  1/15! */
    ps = -1.0 / 6227020800.0 + z * ps;            /* -1/13! */
    ps = 1.0 / 39916800.0 + z * ps;               /*  1/11! */
    ps = -1.0 / 362880.0 + z * ps;                /* -1/9! */
    ps = 1.0 / 5040.0 + z * ps;                   /*  1/7! */
    ps = -1.0 / 120.0 + z * ps;                   /* -1/5! */
    ps = 1.0 / 6.0 + z * ps;                      /*  1/3! */
    const double sx = x - x * (z * ps);
    double pc = 1.0 / 1124000727777607680000.0;   /*  1/22! */
    pc = -1.0 / 2432902008176640000.0 + z * pc;   /* -1/20! */
    pc = 1.0 / 6402373705728000.0 + z * pc;       /*  1/18! */
    pc = -1.0 / 20922789888000.0 + z * pc;        /* -1/16! */
    pc = 1.0 / 87178291200.0 + z * pc;            /*  1/14! */
    pc = -1.0 / 479001600.0 + z * pc;             /* -1/12! */
    pc = 1.0 / 3628800.0 + z * pc;                /*  1/10! */
    pc = -1.0 / 40320.0 + z * pc;                 /* -1/8! */
    pc = 1.0 / 720.0 + z * pc;                    /*  1/6! */
    pc = -1.0 / 24.0 + z * pc;                    /* -1/4! */
    pc = 1.0 / 2.0 + z * pc;                      /*  1/2! */
    const double cx = 1.0 - z * pc;
    switch (((int)n) & 3) {
    case 0: *sn = sx; *cs = cx; break;
    case 1: *sn = cx; *cs = -sx; break;
    case 2: *sn = -sx; *cs = -cx; break;
    default: *sn = -cx; *cs = sx; break;
    }
}

void orc_gaussian_pair(uint64_t seed, uint32_t chain, uint32_t traj, uint32_t stream,
                       uint32_t index, double out[2])
{
    double u[2], sn, cs;
    orc_uniform_pair(seed, chain, traj, stream, index, u);
    double r = sqrt(-2.0 * orc_ln_unit(1.0 - u[0]));
    orc_sincos_turn(u[1], &sn, &cs);
    out[0] = r * cs;
    out[1] = r * sn;
}

/* uniform hot start q in [-pi, pi) */
void orc_random_links(int Lx, int Lt, uint64_t seed, uint32_t chain, double *q)
{
    int nl = 2 * Lx * Lt;
    for (int l = 0; l < nl; ++l) {
        double u[2];
        orc_uniform_pair(seed, chain, 0, STREAM_LINKS, (uint32_t)l, u);
        q[l] = 3.141592653589793 * (2.0 * u[0] - 1.0);
    }
}

/* momenta p ~ N(0, 1), one per link (density exp(-p^2/2) from the kinetic term of Eq. (12)) */
void orc_random_momenta(int Lx, int Lt, uint64_t seed, uint32_t chain, uint32_t traj, double *p)
{
    int nl = 2 * Lx * Lt;
    for (int l = 0; l < nl; ++l) {
        double g[2];
        orc_gaussian_pair(seed, chain, traj, STREAM_MOMENTA, (uint32_t)l, g);
        p[l] = g[0];
    }
}

/* complex Gaussian zeta with density exp(-zeta^dagger zeta): Re, Im ~ N(0, 1/2) */
void orc_random_zeta(int Lx, int Lt, uint64_t seed, uint32_t chain, uint32_t traj, cplx *zeta)
{
    int ns = 2 * Lx * Lt;
    for (int k = 0; k < ns; ++k) {
        double g[2];
        orc_gaussian_pair(seed, chain, traj, STREAM_PSEUDOFERMION, (uint32_t)k, g);
        zeta[k] = g[0] * 0.70710678118654752440 + I * (g[1] * 0.70710678118654752440);
    }
}

double orc_metropolis_uniform(uint64_t seed, uint32_t chain, uint32_t traj)
{
    double u[2];
    orc_uniform_pair(seed, chain, traj, STREAM_METROPOLIS, 0, u);
    return u[0];
}

/* ------------------------------------------------------------------------- */
/* Compensated summation (Neumaier) for energies and their differences       */
/* ------------------------------------------------------------------------- */

typedef struct { double s, c; } ksum;

static void kadd(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}

static double kval(const ksum *k) { return k->s + k->c; }

/* ------------------------------------------------------------------------- */
/* Gauge part: plaquette, Wilson action (Eq. (13)), gauge force (Eq. (16))   */
/* ------------------------------------------------------------------------- */

static cplx link(const double *q, int n, int mu) { return cexp(I * q[2 * n + mu]); }

/*
 * Oriented plaquette P_{mu nu}(n) = U_mu(n) U_nu(n+mu) U_mu^dagger(n+nu) U_nu^dagger(n).
 * P_{01}(n) is the plaquette P(n) of Sec. 3; P_{10}(n) is its complex conjugate.
 */
static cplx plaquette(const double *q, int n, int mu, int nu, int Lx, int Lt)
{
    int n_mu = hop(n, mu, +1, Lx, Lt), n_nu = hop(n, nu, +1, Lx, Lt);
    return link(q, n, mu) * link(q, n_mu, nu) * conj(link(q, n_nu, mu)) * conj(link(q, n, nu));
}

/* S_G = beta * sum_n (1 - Re P(n)), Eq. (13) */
double orc_gauge_action(int Lx, int Lt, double beta, const double *q)
{
    ksum k = {0, 0};
    for (int n = 0; n < Lx * Lt; ++n) kadd(&k, 1.0 - creal(plaquette(q, n, 0, 1, Lx, Lt)));
    return beta * kval(&k);
}

/* average Re P(n) */
double orc_mean_plaquette(int Lx, int Lt, const double *q)
{
    ksum k = {0, 0};
    for (int n = 0; n < Lx * Lt; ++n) kadd(&k, creal(plaquette(q, n, 0, 1, Lx, Lt)));
    return kval(&k) / (double)(Lx * Lt);
}

/*
 * beta g(n, mu) = dS_G/dq_mu(n) = beta Im(P_{mu nu}(n) - P_{mu nu}(n - nu)), nu != mu,
 * Eq. (16), reading P in the mu-first orientation of the plaquettes P_1, P_2 that
 * the paper lists for the force-gradient term C_GG.
 */
void orc_gauge_force(int Lx, int Lt, double beta, const double *q, double *F)
{
    for (int n = 0; n < Lx * Lt; ++n)
        for (int mu = 0; mu < 2; ++mu) {
            int nu = 1 - mu;
            int n_mnu = hop(n, nu, -1, Lx, Lt);
            F[2 * n + mu] = beta * cimag(plaquette(q, n, mu, nu, Lx, Lt) -
                                         plaquette(q, n_mnu, mu, nu, Lx, Lt));
        }
}

/* ------------------------------------------------------------------------- */
/* Wilson-Dirac operator (Sec. 3)                                            */
/* ------------------------------------------------------------------------- */

/* Pauli matrices sigma_1, sigma_2 of Sec. 3, row-major */
static const cplx SIGMA[2][2][2] = {
    {{0, 1}, {1, 0}},
    {{0, -I}, {I, 0}},
};

/* out = (1 + sgn * sigma_mu) v */
static void proj(int mu, int sgn, const cplx v[2], cplx out[2])
{
    for (int a = 0; a < 2; ++a) {
        cplx acc = v[a];
        for (int b = 0; b < 2; ++b) acc += (double)sgn * SIGMA[mu][a][b] * v[b];
        out[a] = acc;
    }
}

/* fermion link: U_mu(n) with the antiperiodic sign on t-links leaving t = Lt-1 */
static cplx flink(const double *q, int n, int mu, int Lx, int Lt)
{
    cplx u = link(q, n, mu);
    if (mu == 1 && n / Lx == Lt - 1) u = -u;
    return u;
}

/*
 * (D psi)(n) = (2 + m0) psi(n)
 *   - 1/2 sum_mu [ (1 - sigma_mu) U_mu(n) psi(n + mu) + (1 + sigma_mu) U_mu^dagger(n - mu) psi(n - mu) ]
 * Sec. 3 (the Wilson-Dirac matrix D_{n,m}).
 */
void orc_dirac(int Lx, int Lt, double m0, const double *q, const cplx *in, cplx *out)
{
    for (int n = 0; n < Lx * Lt; ++n) {
        cplx acc[2] = {(2.0 + m0) * in[2 * n], (2.0 + m0) * in[2 * n + 1]};
        for (int mu = 0; mu < 2; ++mu) {
            int nf = hop(n, mu, +1, Lx, Lt), nb = hop(n, mu, -1, Lx, Lt);
            cplx uf = flink(q, n, mu, Lx, Lt), ub = conj(flink(q, nb, mu, Lx, Lt));
            cplx vf[2] = {uf * in[2 * nf], uf * in[2 * nf + 1]};
            cplx vb[2] = {ub * in[2 * nb], ub * in[2 * nb + 1]};
            cplx pf[2], pb[2];
            proj(mu, -1, vf, pf);
            proj(mu, +1, vb, pb);
            for (int a = 0; a < 2; ++a) acc[a] -= 0.5 * (pf[a] + pb[a]);
        }
        out[2 * n] = acc[0];
        out[2 * n + 1] = acc[1];
    }
}

/*
 * (D psi) at the listed sites only (lexicographic indices sites[0..ns)), out[2*k + s]:
 * the same definition as orc_dirac, evaluated one site at a time for sampled checks on
 * lattices too large to sweep.
 */
void orc_dirac_sites(int Lx, int Lt, double m0, const double *q, const cplx *in, int ns,
                     const long long *sites, cplx *out)
{
    for (int k = 0; k < ns; ++k) {
        int n = (int)sites[k];
        cplx acc[2] = {(2.0 + m0) * in[2 * n], (2.0 + m0) * in[2 * n + 1]};
        for (int mu = 0; mu < 2; ++mu) {
            int nf = hop(n, mu, +1, Lx, Lt), nb = hop(n, mu, -1, Lx, Lt);
            cplx uf = flink(q, n, mu, Lx, Lt), ub = conj(flink(q, nb, mu, Lx, Lt));
            cplx vf[2] = {uf * in[2 * nf], uf * in[2 * nf + 1]};
            cplx vb[2] = {ub * in[2 * nb], ub * in[2 * nb + 1]};
            cplx pf[2], pb[2];
            proj(mu, -1, vf, pf);
            proj(mu, +1, vb, pb);
            for (int a = 0; a < 2; ++a) acc[a] -= 0.5 * (pf[a] + pb[a]);
        }
        out[2 * k] = acc[0];
        out[2 * k + 1] = acc[1];
    }
}

/*
 * D^dagger as the literal conjugate transpose of D_{n,m}: the forward hop carries
 * (1 + sigma_mu) U_mu(n), the backward hop (1 - sigma_mu) U_mu^dagger(n - mu)
 * (sigma_mu is hermitian).  gamma5-hermiticity D^dagger = sigma_3 D sigma_3 is
 * checked by test, not used here.
 */
void orc_dirac_dagger(int Lx, int Lt, double m0, const double *q, const cplx *in, cplx *out)
{
    for (int n = 0; n < Lx * Lt; ++n) {
        cplx acc[2] = {(2.0 + m0) * in[2 * n], (2.0 + m0) * in[2 * n + 1]};
        for (int mu = 0; mu < 2; ++mu) {
            int nf = hop(n, mu, +1, Lx, Lt), nb = hop(n, mu, -1, Lx, Lt);
            cplx uf = flink(q, n, mu, Lx, Lt), ub = conj(flink(q, nb, mu, Lx, Lt));
            cplx vf[2] = {uf * in[2 * nf], uf * in[2 * nf + 1]};
            cplx vb[2] = {ub * in[2 * nb], ub * in[2 * nb + 1]};
            cplx pf[2], pb[2];
            proj(mu, +1, vf, pf);
            proj(mu, -1, vb, pb);
            for (int a = 0; a < 2; ++a) acc[a] -= 0.5 * (pf[a] + pb[a]);
        }
        out[2 * n] = acc[0];
        out[2 * n + 1] = acc[1];
    }
}

/* ------------------------------------------------------------------------- */
/* Conjugate gradient on the normal equations D^dagger D x = phi             */
/* (the solver behind "D^{-1}" in Sec. 3; x0 = 0; relative 2-norm residual)  */
/* ------------------------------------------------------------------------- */

static double dot_re(int ns, const cplx *a, const cplx *b)
{
    ksum k = {0, 0};
    for (int i = 0; i < ns; ++i) kadd(&k, creal(conj(a[i]) * b[i]));
    return kval(&k);
}

static void normal_op(int Lx, int Lt, double m0, const double *q, const cplx *in, cplx *tmp, cplx *out)
{
    orc_dirac(Lx, Lt, m0, q, in, tmp);
    orc_dirac_dagger(Lx, Lt, m0, q, tmp, out);
}

/*
 * Returns the number of iterations, or -1 if max_iter was reached without
 * convergence (x then holds the last iterate).  Stops when ||r_k|| <= tol ||phi||
 * on the recursively updated residual; *true_rel_resid receives
 * ||phi - D^dagger D x|| / ||phi|| recomputed at the end.
 */
int orc_cg(int Lx, int Lt, double m0, const double *q, const cplx *phi, cplx *x, double tol,
           int max_iter, double *true_rel_resid)
{
    int ns = 2 * Lx * Lt;
    cplx *r = malloc(sizeof(cplx) * ns), *p = malloc(sizeof(cplx) * ns);
    cplx *Ap = malloc(sizeof(cplx) * ns), *tmp = malloc(sizeof(cplx) * ns);
    for (int i = 0; i < ns; ++i) { x[i] = 0; r[i] = phi[i]; p[i] = phi[i]; }
    double phi2 = dot_re(ns, phi, phi);
    double rho = phi2;
    int it = 0, converged = (rho <= tol * tol * phi2);
    while (!converged && it < max_iter) {
        normal_op(Lx, Lt, m0, q, p, tmp, Ap);
        double alpha = rho / dot_re(ns, p, Ap);
        for (int i = 0; i < ns; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rho_new = dot_re(ns, r, r);
        ++it;
        if (rho_new <= tol * tol * phi2) { converged = 1; break; }
        double beta = rho_new / rho;
        for (int i = 0; i < ns; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    if (true_rel_resid) {
        normal_op(Lx, Lt, m0, q, x, tmp, Ap);
        for (int i = 0; i < ns; ++i) r[i] = phi[i] - Ap[i];
        *true_rel_resid = phi2 > 0 ? sqrt(dot_re(ns, r, r) / phi2) : 0.0;
    }
    free(r); free(p); free(Ap); free(tmp);
    return converged ? it : -1;
}

/* ------------------------------------------------------------------------- */
/* Fermion action (Eq. (14)) and fermion force (Eqs. (17), (18))             */
/* ------------------------------------------------------------------------- */

/*
 * f(n, mu) = -Im[ chi^dagger(n) (1 - sigma_mu) U_mu(n) xi(n + mu)
 *                 - chi^dagger(n + mu) (1 + sigma_mu) U_mu^dagger(n) xi(n) ]
 * with chi = D^{dagger -1} eta and xi = D^{-1} D^{dagger -1} eta, Eqs. (17)-(18).
 * The fermion link (with the boundary sign) enters; its derivative in q is i times itself.
 */
void orc_fermion_force_chixi(int Lx, int Lt, const double *q, const cplx *chi, const cplx *xi,
                             double *f)
{
    for (int n = 0; n < Lx * Lt; ++n)
        for (int mu = 0; mu < 2; ++mu) {
            int nf = hop(n, mu, +1, Lx, Lt);
            cplx u = flink(q, n, mu, Lx, Lt);
            cplx a[2] = {u * xi[2 * nf], u * xi[2 * nf + 1]};
            cplx b[2] = {conj(u) * xi[2 * n], conj(u) * xi[2 * n + 1]};
            cplx pa[2], pb[2];
            proj(mu, -1, a, pa);
            proj(mu, +1, b, pb);
            cplx term1 = conj(chi[2 * n]) * pa[0] + conj(chi[2 * n + 1]) * pa[1];
            cplx term2 = conj(chi[2 * nf]) * pb[0] + conj(chi[2 * nf + 1]) * pb[1];
            f[2 * n + mu] = -cimag(term1 - term2);
        }
}

/*
 * Solves xi = (D^dagger D)^{-1} phi, forms chi = D xi (= D^{dagger -1} phi) and the
 * force f = dS_F/dq.  Optional outputs: chi, xi, S_F = Re phi^dagger xi.
 * Returns CG iterations or -1 on non-convergence.
 */
int orc_fermion_force(int Lx, int Lt, double m0, const double *q, const cplx *phi, double tol,
                      int max_iter, double *f, cplx *chi_out, cplx *xi_out, double *sf_out)
{
    int ns = 2 * Lx * Lt;
    cplx *xi = malloc(sizeof(cplx) * ns), *chi = malloc(sizeof(cplx) * ns);
    int it = orc_cg(Lx, Lt, m0, q, phi, xi, tol, max_iter, NULL);
    orc_dirac(Lx, Lt, m0, q, xi, chi);
    if (f) orc_fermion_force_chixi(Lx, Lt, q, chi, xi, f);
    if (sf_out) *sf_out = dot_re(ns, phi, xi);
    if (chi_out) memcpy(chi_out, chi, sizeof(cplx) * ns);
    if (xi_out) memcpy(xi_out, xi, sizeof(cplx) * ns);
    free(xi); free(chi);
    return it;
}

/* S_F = phi^dagger (D^dagger D)^{-1} phi, Eq. (14) */
double orc_fermion_action(int Lx, int Lt, double m0, const double *q, const cplx *phi, double tol,
                          int max_iter)
{
    double sf = 0;
    orc_fermion_force(Lx, Lt, m0, q, phi, tol, max_iter, NULL, NULL, NULL, &sf);
    return sf;
}

/* ------------------------------------------------------------------------- */
/* Force-gradient term C (Eqs. (19)-(23))                                    */
/* ------------------------------------------------------------------------- */

/*
 * C_GG, the closed form given in Sec. 3 after Eq. (20):
 *   C_GG(n, mu) = 2 beta^2 [ Im(4 P1 - P2 - P3 - P4 - P5) Re P1
 *                          - Im(4 P2 - P1 - P6 - P7 - P8) Re P2 ],  nu != mu,
 * with the eight plaquettes around the link written out as the paper lists them.
 */
void orc_fg_term_gg(int Lx, int Lt, double beta, const double *q, double *C)
{
    for (int n = 0; n < Lx * Lt; ++n)
        for (int mu = 0; mu < 2; ++mu) {
            int nu = 1 - mu;
            int n_pm = hop(n, mu, +1, Lx, Lt), n_mm = hop(n, mu, -1, Lx, Lt);
            int n_pn = hop(n, nu, +1, Lx, Lt), n_mn = hop(n, nu, -1, Lx, Lt);
            int n_2pm = hop(n_pm, mu, +1, Lx, Lt), n_pm_pn = hop(n_pm, nu, +1, Lx, Lt);
            int n_2pn = hop(n_pn, nu, +1, Lx, Lt), n_mm_pn = hop(n_mm, nu, +1, Lx, Lt);
            int n_mm_mn = hop(n_mm, nu, -1, Lx, Lt), n_2mn = hop(n_mn, nu, -1, Lx, Lt);
            int n_pm_mn = hop(n_pm, nu, -1, Lx, Lt), n_2mn_pm = hop(n_2mn, mu, +1, Lx, Lt);
            int n_pm_mn_pm = hop(n_pm_mn, mu, +1, Lx, Lt);
            cplx P1 = link(q, n, mu) * link(q, n_pm, nu) * conj(link(q, n_pn, mu)) * conj(link(q, n, nu));
            cplx P2 = link(q, n_mn, mu) * link(q, n_pm_mn, nu) * conj(link(q, n, mu)) *
                      conj(link(q, n_mn, nu));
            cplx P3 = link(q, n_pm, mu) * link(q, n_2pm, nu) * conj(link(q, n_pm_pn, mu)) *
                      conj(link(q, n_pm, nu));
            cplx P4 = link(q, n_pn, mu) * link(q, n_pm_pn, nu) * conj(link(q, n_2pn, mu)) *
                      conj(link(q, n_pn, nu));
            cplx P5 = link(q, n_mm, mu) * link(q, n, nu) * conj(link(q, n_mm_pn, mu)) *
                      conj(link(q, n_mm, nu));
            cplx P6 = link(q, n_mm_mn, mu) * link(q, n_mn, nu) * conj(link(q, n_mm, mu)) *
                      conj(link(q, n_mm_mn, nu));
            cplx P7 = link(q, n_2mn, mu) * link(q, n_2mn_pm, nu) * conj(link(q, n_mn, mu)) *
                      conj(link(q, n_2mn, nu));
            cplx P8 = link(q, n_pm_mn, mu) * link(q, n_pm_mn_pm, nu) * conj(link(q, n_pm, mu)) *
                      conj(link(q, n_pm_mn, nu));
            C[2 * n + mu] = 2.0 * beta * beta *
                            (cimag(4.0 * P1 - P2 - P3 - P4 - P5) * creal(P1) -
                             cimag(4.0 * P2 - P1 - P6 - P7 - P8) * creal(P2));
        }
}

/*
 * C_FG, the closed form given in Sec. 3 after C_GG, from the fermion force f:
 *   C_FG(n, mu) = 2 beta [ (f(n,mu) + f(n+mu,nu) - f(n+nu,mu) - f(n,nu)) Re P1
 *                        + (f(n,mu) - f(n+mu-nu,nu) - f(n-nu,mu) + f(n-nu,nu)) Re P2 ].
 */
void orc_fg_term_fg(int Lx, int Lt, double beta, const double *q, const double *f, double *C)
{
    for (int n = 0; n < Lx * Lt; ++n)
        for (int mu = 0; mu < 2; ++mu) {
            int nu = 1 - mu;
            int n_pm = hop(n, mu, +1, Lx, Lt), n_pn = hop(n, nu, +1, Lx, Lt);
            int n_mn = hop(n, nu, -1, Lx, Lt), n_pm_mn = hop(n_pm, nu, -1, Lx, Lt);
            double reP1 = creal(plaquette(q, n, mu, nu, Lx, Lt));
            double reP2 = creal(plaquette(q, n_mn, mu, nu, Lx, Lt));
            double a = f[2 * n + mu] + f[2 * n_pm + nu] - f[2 * n_pn + mu] - f[2 * n + nu];
            double b = f[2 * n + mu] - f[2 * n_pm_mn + nu] - f[2 * n_mn + mu] + f[2 * n_mn + nu];
            C[2 * n + mu] = 2.0 * beta * (a * reP1 + b * reP2);
        }
}

/*
 * The two non-zero site entries of w_{1,m,nu} (kind 1) or w_{2,m,nu} (kind 2), Sec. 3
 * after Eq. (21):
 *   w_{1,m,nu} = dD^dagger/dq_nu(m) chi:  at m + nu:  (i/2)(1 - sigma_nu) U_nu^dagger(m) chi(m)
 *                                         at m:      -(i/2)(1 + sigma_nu) U_nu(m) chi(m + nu)
 *   w_{2,m,nu} = dD/dq_nu(m) xi:          at m:      -(i/2)(1 - sigma_nu) U_nu(m) xi(m + nu)
 *                                         at m + nu:  (i/2)(1 + sigma_nu) U_nu^dagger(m) xi(m)
 * U is the fermion link (with the boundary sign).  at_m and at_mnu receive the spinors at
 * sites m and m + nu.
 */
static void w_entries(int kind, int Lx, int Lt, const double *q, int m, int nu, const cplx *psi,
                      cplx at_m[2], cplx at_mnu[2])
{
    int m_nu = hop(m, nu, +1, Lx, Lt);
    cplx u = flink(q, m, nu, Lx, Lt);
    cplx a[2] = {u * psi[2 * m_nu], u * psi[2 * m_nu + 1]};  /* U_nu(m) psi(m + nu) */
    cplx b[2] = {conj(u) * psi[2 * m], conj(u) * psi[2 * m + 1]}; /* U_nu^dagger(m) psi(m) */
    cplx pa[2], pb[2];
    if (kind == 1) {
        proj(nu, +1, a, pa);
        proj(nu, -1, b, pb);
        for (int s = 0; s < 2; ++s) { at_m[s] = -0.5 * I * pa[s]; at_mnu[s] = 0.5 * I * pb[s]; }
    } else {
        proj(nu, -1, a, pa);
        proj(nu, +1, b, pb);
        for (int s = 0; s < 2; ++s) { at_m[s] = -0.5 * I * pa[s]; at_mnu[s] = 0.5 * I * pb[s]; }
    }
}

/* D^{-1} y = (D^dagger D)^{-1} D^dagger y and D^{dagger -1} y = D (D^dagger D)^{-1} y */
static int solve_D(int Lx, int Lt, double m0, const double *q, const cplx *y, cplx *out,
                   int dagger, double tol, int max_iter)
{
    int ns = 2 * Lx * Lt;
    cplx *rhs = malloc(sizeof(cplx) * ns), *sol = malloc(sizeof(cplx) * ns);
    if (dagger) memcpy(rhs, y, sizeof(cplx) * ns);
    else orc_dirac_dagger(Lx, Lt, m0, q, y, rhs);
    int it = orc_cg(Lx, Lt, m0, q, rhs, sol, tol, max_iter, NULL);
    if (dagger) orc_dirac(Lx, Lt, m0, q, sol, out);
    else memcpy(out, sol, sizeof(cplx) * ns);
    free(rhs); free(sol);
    return it;
}

/*
 * The fermion-action part of C with weight vector v, Eqs. (22) and (23):
 *   Z_1 = D^{dagger -1} sum_{m,nu} w_{1,m,nu} v(m,nu),
 *   Z_2 = D^{-1} ( sum_{m,nu} w_{2,m,nu} v(m,nu) + Z_1 ),
 *   C(n,mu) = 4 Re[ Z_1^dagger w_{2,n,mu} + w_{1,n,mu}^dagger Z_2
 *                   - chi^dagger (d^2 D / dq_mu(n)^2) xi v(n,mu) ].
 * v = f gives C_FF; v = beta g (the gauge force) gives C_GF (the remark after Eq. (23)).
 * chi and xi are those of Eq. (18) at the same links.  d^2 D/dq_mu(n)^2 has the entries
 * (1/2)(1 - sigma_mu) U_mu(n) at (n, n+mu) and (1/2)(1 + sigma_mu) U_mu^dagger(n) at
 * (n+mu, n) (each link enters D through exp(i q), so two derivatives give -1 times the
 * hopping entry).  Two inversions (Z_1 and Z_2).  Returns the CG iterations or -1.
 */
int orc_fg_term_fermion(int Lx, int Lt, double m0, const double *q, const cplx *chi,
                        const cplx *xi, const double *v, double tol, int max_iter, double *C)
{
    int V = Lx * Lt, ns = 2 * V;
    cplx *W1 = calloc(ns, sizeof(cplx)), *W2 = calloc(ns, sizeof(cplx));
    cplx *Z1 = malloc(sizeof(cplx) * ns), *Z2 = malloc(sizeof(cplx) * ns);
    cplx *y = malloc(sizeof(cplx) * ns);
    for (int m = 0; m < V; ++m)
        for (int nu = 0; nu < 2; ++nu) {
            int m_nu = hop(m, nu, +1, Lx, Lt);
            cplx e0[2], e1[2];
            w_entries(1, Lx, Lt, q, m, nu, chi, e0, e1);
            for (int s = 0; s < 2; ++s) {
                W1[2 * m + s] += v[2 * m + nu] * e0[s];
                W1[2 * m_nu + s] += v[2 * m + nu] * e1[s];
            }
            w_entries(2, Lx, Lt, q, m, nu, xi, e0, e1);
            for (int s = 0; s < 2; ++s) {
                W2[2 * m + s] += v[2 * m + nu] * e0[s];
                W2[2 * m_nu + s] += v[2 * m + nu] * e1[s];
            }
        }
    int it1 = solve_D(Lx, Lt, m0, q, W1, Z1, 1, tol, max_iter);
    for (int k = 0; k < ns; ++k) y[k] = W2[k] + Z1[k];
    int it2 = solve_D(Lx, Lt, m0, q, y, Z2, 0, tol, max_iter);
    for (int n = 0; n < V; ++n)
        for (int mu = 0; mu < 2; ++mu) {
            int n_mu = hop(n, mu, +1, Lx, Lt);
            cplx w1m[2], w1p[2], w2m[2], w2p[2];
            w_entries(1, Lx, Lt, q, n, mu, chi, w1m, w1p);
            w_entries(2, Lx, Lt, q, n, mu, xi, w2m, w2p);
            cplx acc = 0;
            for (int s = 0; s < 2; ++s) {
                acc += conj(Z1[2 * n + s]) * w2m[s] + conj(Z1[2 * n_mu + s]) * w2p[s];
                acc += conj(w1m[s]) * Z2[2 * n + s] + conj(w1p[s]) * Z2[2 * n_mu + s];
            }
            cplx u = flink(q, n, mu, Lx, Lt);
            cplx a[2] = {u * xi[2 * n_mu], u * xi[2 * n_mu + 1]};
            cplx b[2] = {conj(u) * xi[2 * n], conj(u) * xi[2 * n + 1]};
            cplx pa[2], pb[2];
            proj(mu, -1, a, pa);
            proj(mu, +1, b, pb);
            cplx d2 = 0;
            for (int s = 0; s < 2; ++s)
                d2 += conj(chi[2 * n + s]) * 0.5 * pa[s] + conj(chi[2 * n_mu + s]) * 0.5 * pb[s];
            C[2 * n + mu] = 4.0 * creal(acc - d2 * v[2 * n + mu]);
        }
    free(W1); free(W2); free(Z1); free(Z2); free(y);
    if (it1 < 0 || it2 < 0) return -1;
    return it1 + it2;
}

/*
 * C of Eq. (19) for the force set `which` (0: S_G, 1: S_F, 2: S_G + S_F), assembled from
 * the parts of Eq. (20): C_GG; C_FF; C_GG + C_FG + C_GF + C_FF.  chi, xi and the fermion
 * force f belong to the links q (unused when fermions == 0, which drops the fermion
 * parts).  cnt accumulates [0] CG solves, [1] CG iterations, [2] inversions of D or
 * D^dagger counted as in Sec. 3 (Z_1 and Z_2 one each), [3] failures.
 */
static void fg_term_from(int Lx, int Lt, double beta, double m0, const double *q, int which,
                         int fermions, const cplx *chi, const cplx *xi, const double *f,
                         double tol, int max_iter, double *C, long cnt[4])
{
    int nl = 2 * Lx * Lt;
    double *part = malloc(sizeof(double) * nl), *g = malloc(sizeof(double) * nl);
    for (int l = 0; l < nl; ++l) C[l] = 0;
    if (which == 0 || which == 2) {
        orc_fg_term_gg(Lx, Lt, beta, q, part);
        for (int l = 0; l < nl; ++l) C[l] += part[l];
    }
    if ((which == 1 || which == 2) && fermions) {
        if (which == 2) {
            orc_fg_term_fg(Lx, Lt, beta, q, f, part); /* C_FG */
            for (int l = 0; l < nl; ++l) C[l] += part[l];
            orc_gauge_force(Lx, Lt, beta, q, g); /* C_GF: f replaced by beta g */
            int it = orc_fg_term_fermion(Lx, Lt, m0, q, chi, xi, g, tol, max_iter, part);
            cnt[0] += 2; cnt[2] += 2;
            if (it < 0) { cnt[3]++; it = 2 * max_iter; }
            cnt[1] += it;
            for (int l = 0; l < nl; ++l) C[l] += part[l];
        }
        int it = orc_fg_term_fermion(Lx, Lt, m0, q, chi, xi, f, tol, max_iter, part); /* C_FF */
        cnt[0] += 2; cnt[2] += 2;
        if (it < 0) { cnt[3]++; it = 2 * max_iter; }
        cnt[1] += it;
        for (int l = 0; l < nl; ++l) C[l] += part[l];
    }
    free(part); free(g);
}

/*
 * C of Eq. (19) at links q for the force set `which` (see fg_term_from), solving for chi
 * and xi first (Eq. (18); two inversions).  counters (optional, 3 entries): CG solves, CG
 * iterations, inversions.  Returns 0 or -3 if a solve did not converge.
 */
int orc_force_gradient_term(int Lx, int Lt, double beta, double m0, const double *q,
                            const cplx *phi, int which, double tol, int max_iter, double *C,
                            long *counters)
{
    int nl = 2 * Lx * Lt, ns = 2 * Lx * Lt;
    long cnt[4] = {0, 0, 0, 0};
    double *f = calloc(nl, sizeof(double));
    cplx *chi = calloc(ns, sizeof(cplx)), *xi = calloc(ns, sizeof(cplx));
    if (which == 1 || which == 2) {
        int it = orc_fermion_force(Lx, Lt, m0, q, phi, tol, max_iter, f, chi, xi, NULL);
        cnt[0]++; cnt[2] += 2;
        if (it < 0) { cnt[3]++; it = max_iter; }
        cnt[1] += it;
    }
    fg_term_from(Lx, Lt, beta, m0, q, which, 1, chi, xi, f, tol, max_iter, C, cnt);
    if (counters) { counters[0] = cnt[0]; counters[1] = cnt[1]; counters[2] = cnt[2]; }
    free(f); free(chi); free(xi);
    return cnt[3] ? -3 : 0;
}

/* ------------------------------------------------------------------------- */
/* Molecular dynamics (Sec. 2.1, 2.2)                                        */
/* ------------------------------------------------------------------------- */

enum {
    SCHEME_LEAPFROG = 0,          /* Eq. (3)  */
    SCHEME_OMELYAN_5STAGE = 1,    /* Eq. (4)  */
    SCHEME_FORCE_GRADIENT = 2,    /* Eq. (5), force-gradient term via the shifted force */
    SCHEME_NESTED_FG = 3,         /* Eq. (10) */
    SCHEME_ADAPTED_NESTED_FG = 4, /* Eq. (11) */
    SCHEME_NESTED_LEAPFROG = 5,   /* Eq. (8)  */
    SCHEME_NESTED_5STAGE = 6,     /* Eq. (9)  */
    SCHEME_OMELYAN_11STAGE = 7,   /* Eq. (6)  */
};

/*
 * sigma, eta, lambda, theta of the 11-stage decomposition, Eq. (6): the fourth-order set
 * of Omelyan, Mryglod and Folk (2003), their Eq. (71).
 */
#define OMF_SIGMA 0.08398315262876693
#define OMF_ETA 0.2539785108410595
#define OMF_LAMBDA 0.6822365335719091
#define OMF_THETA (-0.03230286765269967)

/* stage kinds recorded in the trace */
enum {
    ST_A = 0,      /* e^{eps A}: q += eps p */
    ST_B = 1,      /* kick with the full force F_G + F_F */
    ST_BG = 2,     /* kick with the gauge force only (fast part B_1) */
    ST_BF = 3,     /* kick with the fermion force only (slow part B_2) */
    ST_BT = 4,     /* force-gradient kick with the full force */
    ST_BTG = 5,    /* force-gradient kick with the gauge force */
    ST_BTF = 6,    /* force-gradient kick with the fermion force */
};

#define FLAG_QUENCHED 1 /* drop S_F entirely (pure gauge HMC, used for exact-plaquette tests) */
#define FLAG_FG_EXACT 2 /* force-gradient kicks use the exact C of Eqs. (19)-(23), not the shift */

typedef struct {
    int Lx, Lt, flags;
    double beta, m0, tol;
    int max_iter;
    double *q, *p;
    const cplx *phi;
    double *F, *F2, *qs; /* scratch: force, shifted force, saved links */
    double *ff, *C;      /* fermion force of the last force evaluation; force-gradient term */
    cplx *chi, *xi;      /* chi, xi (Eq. (18)) of the last fermion-force evaluation */
    /* counters */
    long n_solves, n_cg_iters, n_dinv;
    int failed;
    /* optional stage trace */
    int *trace_kind;
    double *trace_eps;
    int trace_cap, trace_len;
} md_state;

static void trace(md_state *s, int kind, double eps)
{
    if (s->trace_kind && s->trace_len < s->trace_cap) {
        s->trace_kind[s->trace_len] = kind;
        s->trace_eps[s->trace_len] = eps;
    }
    s->trace_len++;
}

/* F = dS_G/dq (+ dS_F/dq); which: 0 gauge, 1 fermion, 2 total */
static void force(md_state *s, int which, const double *q, double *F)
{
    int nl = 2 * s->Lx * s->Lt;
    int use_f = !(s->flags & FLAG_QUENCHED);
    if (which == 0 || which == 2) orc_gauge_force(s->Lx, s->Lt, s->beta, q, F);
    else for (int l = 0; l < nl; ++l) F[l] = 0;
    if ((which == 1 || which == 2) && use_f) {
        int it = orc_fermion_force(s->Lx, s->Lt, s->m0, q, s->phi, s->tol, s->max_iter, s->ff,
                                   s->chi, s->xi, NULL);
        s->n_solves++;
        s->n_dinv += 2;
        if (it < 0) { s->failed = 1; it = s->max_iter; }
        s->n_cg_iters += it;
        for (int l = 0; l < nl; ++l) F[l] += s->ff[l];
    }
}

/* e^{eps A}: U' = exp(i P eps) U, i.e. q' = q + eps p (Sec. 2.1) */
static void stage_A(md_state *s, double eps)
{
    int nl = 2 * s->Lx * s->Lt;
    for (int l = 0; l < nl; ++l) s->q[l] += eps * s->p[l];
    trace(s, ST_A, eps);
}

/* e^{eps B}: p' = p - eps F (Sec. 2.1; the momenta are real for U(1)) */
static void stage_B(md_state *s, int which, double eps)
{
    int nl = 2 * s->Lx * s->Lt;
    force(s, which, s->q, s->F);
    for (int l = 0; l < nl; ++l) s->p[l] -= eps * s->F[l];
    trace(s, which == 0 ? ST_BG : which == 1 ? ST_BF : ST_B, eps);
}

/*
 * Force-gradient kick e^{eps B + c h^3 C} with eps = 2h/3 and the force-gradient
 * term approximated through a force evaluated at shifted links (Sec. 2.2, the
 * Taylor-expansion variant): the kick is p' = p - eps F(q - (h^2/24) F(q)), which
 * equals p - eps F + (h^3/72) C + O(h^5) with C = grad |F|^2 of Eq. (19).  The
 * links are restored afterwards.  `h` is the step of the level the kick belongs to.
 */
static void stage_B_fg_shift(md_state *s, int which, double eps, double h)
{
    int nl = 2 * s->Lx * s->Lt;
    force(s, which, s->q, s->F);
    for (int l = 0; l < nl; ++l) s->qs[l] = s->q[l] - (h * h / 24.0) * s->F[l];
    force(s, which, s->qs, s->F2);
    for (int l = 0; l < nl; ++l) s->p[l] -= eps * s->F2[l];
    trace(s, which == 0 ? ST_BTG : which == 1 ? ST_BTF : ST_BT, eps);
}

/*
 * The same kick with the exact force-gradient term of Eq. (5): p' = p - eps F + (h^3/72) C
 * with C from Eqs. (19)-(23) for the same force set (C_GG for the gauge force alone, C_FF
 * for the fermion force alone as the nested schemes require, all four parts for the full
 * force).
 */
static void stage_B_fg_exact(md_state *s, int which, double eps, double h)
{
    int nl = 2 * s->Lx * s->Lt;
    long cnt[4] = {0, 0, 0, 0};
    force(s, which, s->q, s->F);
    fg_term_from(s->Lx, s->Lt, s->beta, s->m0, s->q, which, !(s->flags & FLAG_QUENCHED), s->chi,
                 s->xi, s->ff, s->tol, s->max_iter, s->C, cnt);
    s->n_solves += cnt[0];
    s->n_cg_iters += cnt[1];
    s->n_dinv += cnt[2];
    if (cnt[3]) s->failed = 1;
    for (int l = 0; l < nl; ++l) s->p[l] += -eps * s->F[l] + (h * h * h / 72.0) * s->C[l];
    trace(s, which == 0 ? ST_BTG : which == 1 ? ST_BTF : ST_BT, eps);
}

static void stage_B_fg(md_state *s, int which, double eps, double h)
{
    if (s->flags & FLAG_FG_EXACT) stage_B_fg_exact(s, which, eps, h);
    else stage_B_fg_shift(s, which, eps, h);
}

/* Delta_1(s)_M = (e^{s/(2M) B_1} e^{s/M A} e^{s/(2M) B_1})^M, the inner leapfrog of Eq. (8) */
static void inner_leapfrog(md_state *st, double s, int M)
{
    for (int k = 0; k < M; ++k) {
        stage_B(st, 0, s / (2.0 * M));
        stage_A(st, s / M);
        stage_B(st, 0, s / (2.0 * M));
    }
}

/* Delta_2(s)_M of Eq. (10): M inner 5-stage force-gradient steps of size s/M on A + B_1 */
static void inner_fg(md_state *st, double s, int M)
{
    double hm = s / M;
    for (int k = 0; k < M; ++k) {
        stage_B(st, 0, hm / 6.0);
        stage_A(st, hm / 2.0);
        stage_B_fg(st, 0, 2.0 * hm / 3.0, hm);
        stage_A(st, hm / 2.0);
        stage_B(st, 0, hm / 6.0);
    }
}

/* one outer step of size h */
static void md_step(md_state *s, int scheme, double h, int M)
{
    switch (scheme) {
    case SCHEME_LEAPFROG: /* Eq. (3) */
        stage_B(s, 2, h / 2.0);
        stage_A(s, h);
        stage_B(s, 2, h / 2.0);
        break;
    case SCHEME_OMELYAN_5STAGE: /* Eq. (4) */
        stage_B(s, 2, h / 6.0);
        stage_A(s, h / 2.0);
        stage_B(s, 2, 2.0 * h / 3.0);
        stage_A(s, h / 2.0);
        stage_B(s, 2, h / 6.0);
        break;
    case SCHEME_FORCE_GRADIENT: /* Eq. (5) */
        stage_B(s, 2, h / 6.0);
        stage_A(s, h / 2.0);
        stage_B_fg(s, 2, 2.0 * h / 3.0, h);
        stage_A(s, h / 2.0);
        stage_B(s, 2, h / 6.0);
        break;
    case SCHEME_NESTED_FG: /* Eq. (10) */
        stage_B(s, 1, h / 6.0);
        inner_fg(s, h / 2.0, M);
        stage_B_fg(s, 1, 2.0 * h / 3.0, h);
        inner_fg(s, h / 2.0, M);
        stage_B(s, 1, h / 6.0);
        break;
    case SCHEME_ADAPTED_NESTED_FG: /* Eq. (11) */
        stage_B(s, 1, h / 6.0);
        inner_leapfrog(s, h / 2.0, M);
        stage_B_fg(s, 1, 2.0 * h / 3.0, h);
        inner_leapfrog(s, h / 2.0, M);
        stage_B(s, 1, h / 6.0);
        break;
    case SCHEME_NESTED_LEAPFROG: /* Eq. (8): the inner leap-frog spans the whole step h */
        stage_B(s, 1, h / 2.0);
        inner_leapfrog(s, h, M);
        stage_B(s, 1, h / 2.0);
        break;
    case SCHEME_NESTED_5STAGE: /* Eq. (9) */
        stage_B(s, 1, h / 6.0);
        inner_leapfrog(s, h / 2.0, M);
        stage_B(s, 1, 2.0 * h / 3.0);
        inner_leapfrog(s, h / 2.0, M);
        stage_B(s, 1, h / 6.0);
        break;
    case SCHEME_OMELYAN_11STAGE: { /* Eq. (6) */
        double bm = (1.0 - 2.0 * (OMF_LAMBDA + OMF_SIGMA)) / 2.0, am = 1.0 - 2.0 * (OMF_THETA + OMF_ETA);
        stage_B(s, 2, OMF_SIGMA * h);
        stage_A(s, OMF_ETA * h);
        stage_B(s, 2, OMF_LAMBDA * h);
        stage_A(s, OMF_THETA * h);
        stage_B(s, 2, bm * h);
        stage_A(s, am * h);
        stage_B(s, 2, bm * h);
        stage_A(s, OMF_THETA * h);
        stage_B(s, 2, OMF_LAMBDA * h);
        stage_A(s, OMF_ETA * h);
        stage_B(s, 2, OMF_SIGMA * h);
        break;
    }
    }
}

/*
 * Integrates Hamilton's equations (Eq. (2)) for a trajectory of length tau with
 * n_outer steps h = tau / n_outer; n_inner = M is the number of inner steps in
 * each inner call of the nested schemes.  q and p are updated in place.
 * counters[0] = CG solves, counters[1] = total CG iterations, counters[2] = stages
 * recorded, counters[3] = inversions of D or D^dagger counted as in Sec. 3 (two per
 * fermion-force evaluation, one each for Z_1 and Z_2).  Returns 0, or -3 if a solve did not converge.
 */
int orc_md_integrate(int Lx, int Lt, double beta, double m0, int scheme, double tau, int n_outer,
                     int n_inner, double tol, int max_iter, int flags, double *q, double *p,
                     const cplx *phi, long *counters, int *trace_kind, double *trace_eps,
                     int trace_cap)
{
    int nl = 2 * Lx * Lt;
    md_state s;
    memset(&s, 0, sizeof(s));
    s.Lx = Lx; s.Lt = Lt; s.flags = flags; s.beta = beta; s.m0 = m0; s.tol = tol;
    s.max_iter = max_iter; s.q = q; s.p = p; s.phi = phi;
    s.F = malloc(sizeof(double) * nl);
    s.F2 = malloc(sizeof(double) * nl);
    s.qs = malloc(sizeof(double) * nl);
    s.ff = calloc(nl, sizeof(double));
    s.C = malloc(sizeof(double) * nl);
    s.chi = calloc(nl, sizeof(cplx));
    s.xi = calloc(nl, sizeof(cplx));
    s.trace_kind = trace_kind; s.trace_eps = trace_eps; s.trace_cap = trace_cap;
    double h = tau / n_outer;
    for (int k = 0; k < n_outer; ++k) md_step(&s, scheme, h, n_inner);
    free(s.F); free(s.F2); free(s.qs); free(s.ff); free(s.C); free(s.chi); free(s.xi);
    if (counters) {
        counters[0] = s.n_solves;
        counters[1] = s.n_cg_iters;
        counters[2] = s.trace_len;
        counters[3] = s.n_dinv;
    }
    return s.failed ? -3 : 0;
}

/* ------------------------------------------------------------------------- */
/* HMC update (Sec. 2.1)                                                     */
/* ------------------------------------------------------------------------- */

/*
 * One HMC trajectory from links q (updated in place on acceptance):
 *   p ~ N(0,1) (stream 1), zeta complex Gaussian (stream 2), phi = D^dagger zeta, so that
 *   phi is distributed as exp(-S_F) of Eq. (14) and S_F(U0) = zeta^dagger zeta exactly;
 *   molecular dynamics to (q', p'); Delta H = H(q', p') - H(q, p) summed as a sum of
 *   per-term differences; accept iff Delta H <= 0 or u < exp(-Delta H) with u from stream 3.
 * info[0] = Delta H, info[1] = accepted (0/1), info[2] = mean plaquette after the update,
 * info[3] = fermion solves, info[4] = total CG iterations, info[5] = H0, info[6] = H1,
 * info[7] = Metropolis uniform, info[8] = inversions of D or D^dagger in the molecular
 * dynamics (as counted by orc_md_integrate).
 * Returns 0, -3 (CG failure: trajectory rejected) or -5 (non-finite Delta H: rejected).
 */
int orc_hmc_trajectory(int Lx, int Lt, double beta, double m0, uint64_t seed, uint32_t chain,
                       uint32_t traj, int scheme, double tau, int n_outer, int n_inner, double tol,
                       int max_iter, int flags, double *q, double *info)
{
    int V = Lx * Lt, nl = 2 * V, ns = 2 * V;
    double *q0 = malloc(sizeof(double) * nl), *p = malloc(sizeof(double) * nl);
    double *p0 = malloc(sizeof(double) * nl);
    cplx *zeta = malloc(sizeof(cplx) * ns), *phi = malloc(sizeof(cplx) * ns);
    cplx *xi = malloc(sizeof(cplx) * ns);
    memcpy(q0, q, sizeof(double) * nl);
    orc_random_momenta(Lx, Lt, seed, chain, traj, p);
    memcpy(p0, p, sizeof(double) * nl);
    int quenched = flags & FLAG_QUENCHED;
    if (!quenched) {
        orc_random_zeta(Lx, Lt, seed, chain, traj, zeta);
        orc_dirac_dagger(Lx, Lt, m0, q, zeta, phi);
    } else {
        for (int k = 0; k < ns; ++k) phi[k] = 0;
    }
    long counters[4] = {0, 0, 0, 0};
    int rc = orc_md_integrate(Lx, Lt, beta, m0, scheme, tau, n_outer, n_inner, tol, max_iter,
                              flags, q, p, phi, counters, NULL, NULL, 0);
    double sf1 = 0, sf0 = 0;
    if (!quenched) {
        int it = orc_cg(Lx, Lt, m0, q, phi, xi, tol, max_iter, NULL);
        counters[0]++;
        if (it < 0) { rc = -3; it = max_iter; }
        counters[1] += it;
        sf1 = dot_re(ns, phi, xi);
        sf0 = dot_re(ns, zeta, zeta);
    }
    /* Delta H as a sum of differences (Eq. (12)) */
    ksum dk = {0, 0}, dg = {0, 0};
    ksum h0 = {0, 0}, h1 = {0, 0};
    for (int l = 0; l < nl; ++l) {
        kadd(&dk, 0.5 * (p[l] - p0[l]) * (p[l] + p0[l]));
        kadd(&h0, 0.5 * p0[l] * p0[l]);
        kadd(&h1, 0.5 * p[l] * p[l]);
    }
    for (int n = 0; n < V; ++n) {
        double c0 = creal(plaquette(q0, n, 0, 1, Lx, Lt)), c1 = creal(plaquette(q, n, 0, 1, Lx, Lt));
        kadd(&dg, c0 - c1);
        kadd(&h0, beta * (1.0 - c0));
        kadd(&h1, beta * (1.0 - c1));
    }
    double dH = kval(&dk) + beta * kval(&dg) + (sf1 - sf0);
    kadd(&h0, sf0);
    kadd(&h1, sf1);
    double u = orc_metropolis_uniform(seed, chain, traj);
    int accept = 0;
    if (rc == 0 && !isfinite(dH)) rc = -5;
    if (rc == 0) accept = (dH <= 0.0) || (u < exp(-dH));
    if (!accept) memcpy(q, q0, sizeof(double) * nl);
    if (info) {
        info[0] = dH; info[1] = accept; info[2] = orc_mean_plaquette(Lx, Lt, q);
        info[3] = (double)counters[0]; info[4] = (double)counters[1];
        info[5] = kval(&h0); info[6] = kval(&h1); info[7] = u; info[8] = (double)counters[3];
    }
    free(q0); free(p); free(p0); free(zeta); free(phi); free(xi);
    return rc;
}
