/*
 * VEGAS+ iteration -- CPU reference oracle (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the slow, obviously-correct, single-threaded FP64 statement of
 * what one VEGAS+ iteration computes.  It exists to check the HIP path; only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * it.  It shares no code, header, constant table or helper with the HIP
 * library, and the library never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (oracle/build.py).
 * Contraction is off so that every a*b+c below rounds twice unless it is
 * written as fma(); the HIP side follows the same written order.
 *
 * Paper: Tolotti et al., "cuVegas", arXiv:2408.09229.  Citations name the
 * section / equation / algorithm.  Where the paper is silent the reading is
 * marked READING and listed in the design notes.
 *
 *   Sec. 2.1.1 Eq. (1)-(4)  importance-sampling map, J(y) = N_g * dx_{i(y)}
 *   Sec. 2.1.2 Eq. (5)-(7)  stratified sampling, I = sum dI_h,
 *                           sigma^2 = sum sigma_h^2 / n_h, n_h ~ sigma_h^beta
 *   Sec. 2.1.3 Eq. (8)-(9)  inverse-variance combination of iterations
 *   Sec. 3.2 Alg. 1, Alg. 2 main loop and VegasFill
 *   Sec. 4.1 Tab. 2         default parameters (alpha, beta, N_g)
 *   Sec. 4.1 Tab. 3         test integrands
 *
 * Parity status per function is stated beside it ("pinned by ...").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random        */
/* numbers: as easy as 1, 2, 3").  Replaces the paper's per-thread XORWOW     */
/* states (Sec. 3.3.2) with a counter-based stream: the words of sample k do   */
/* not depend on which thread draws them.                                     */
/* Pinned by the published known-answer vectors and by rocRAND on the GPU.    */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    /* One S-box round: two 32x32->64 products, then xor/permute. */
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

ORC_EXPORT void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                                  uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {               /* Weyl key schedule between rounds */
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* The random word for (iteration t, sample k, dimension d, instance inst):
 * counter = (k mod 2^32, k div 2^32, t, (inst << 8) | floor(d/4)),
 * key = (seed mod 2^32, seed div 2^32), output word d mod 4.  READING. */
ORC_EXPORT uint32_t orc_word(uint64_t seed, uint32_t inst, uint32_t t,
                             uint64_t k, int d)
{
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), t,
                       (inst << 8) | (uint32_t)(d / 4)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[d % 4];
}

/* ------------------------------------------------------------------------ */
/* Deterministic log / exp from IEEE +,-,*,/, fma, frexp, ldexp only.          */
/* Used by the map damping (Sec. 2.1.1) and the general-beta allocation        */
/* power (Sec. 2.1.2), so that map and allocation updates are reproducible     */
/* bit for bit on any machine that follows the same written order.             */
/* Pinned against mpmath (|err| <= 2 ulp).                                     */
/* ------------------------------------------------------------------------ */
/* ln 2 split so that e*LN2_HI is exact for |e| < 2^11 (low 11 mantissa bits
 * of the nearest double cleared); LN2_LO = ln 2 - LN2_HI rounded. */
static const double LN2_HI  = 0x1.62e42fefa3800p-1;
static const double LN2_LO  = 0x1.ef35793c76730p-45;
static const double INV_LN2 = 0x1.71547652b82fep+0;   /* 1/ln 2 rounded */
static const double SQRT_HALF = 0x1.6a09e667f3bcdp-1;

ORC_EXPORT double orc_det_log(double x)
{
    if (x != x || x < 0.0) return NAN;
    if (x == 0.0) return -INFINITY;
    if (isinf(x)) return x;
    int e;
    double m = frexp(x, &e);               /* x = m 2^e, m in [0.5, 1) */
    if (m < SQRT_HALF) { m = 2.0 * m; e -= 1; }   /* m in [sqrt(1/2), sqrt 2) */
    double s = (m - 1.0) / (m + 1.0);      /* ln m = 2 atanh(s) */
    double z = s * s;
    /* atanh(s)/s = sum_k z^k/(2k+1), k = 0..11, Horner with fma. */
    double p = 1.0 / 23.0;
    for (int k = 10; k >= 0; --k) p = fma(p, z, 1.0 / (double)(2 * k + 1));
    double de = (double)e;
    double t1 = de * LN2_HI;
    double t2 = de * LN2_LO;
    double t4 = (2.0 * s) * p;
    return t1 + (t2 + t4);
}

ORC_EXPORT double orc_det_exp(double x)
{
    if (x != x) return x;
    if (x > 709.8) return INFINITY;
    if (x < -745.2) return 0.0;
    double kd = nearbyint(x * INV_LN2);    /* round half to even */
    double r = (x - kd * LN2_HI) - kd * LN2_LO;
    /* exp(r) = sum_{j=0..13} r^j / j!, Horner with fma. */
    double fact[14];
    fact[0] = 1.0;
    for (int j = 1; j < 14; ++j) fact[j] = fact[j - 1] * (double)j; /* exact */
    double p = 1.0 / fact[13];
    for (int j = 12; j >= 0; --j) p = fma(p, r, 1.0 / fact[j]);
    return ldexp(p, (int)kd);
}

/* ------------------------------------------------------------------------ */
/* Strata (Sec. 2.1.2).  READING: N_st is the largest m >= 1 with              */
/* 4 m^D <= N_ev (integer arithmetic), lowered until R = N_ev - n_min N_c >= 0 */
/* Pinned by brute force over small (D, N_ev).                                 */
/* ------------------------------------------------------------------------ */
static int pow_le(uint64_t m, int D, uint64_t limit, uint64_t* out)
{   /* m^D <= limit ? (without overflow) */
    uint64_t v = 1;
    for (int d = 0; d < D; ++d) {
        if (m != 0 && v > limit / m) return 0;
        v *= m;
    }
    if (v > limit) return 0;
    if (out) *out = v;
    return 1;
}

ORC_EXPORT int orc_strata(int64_t n_eval, int D, int n_min, int n_strat_req,
                          int64_t* n_strat, int64_t* n_cubes, int64_t* R)
{
    if (D < 1 || n_eval < 1 || n_min < 2) return -1;
    uint64_t m;
    if (n_strat_req > 0) {
        m = (uint64_t)n_strat_req;
    } else {
        m = 1;
        while (pow_le(m + 1, D, (uint64_t)n_eval / 4, NULL)) ++m;
    }
    uint64_t nc = 0;
    for (;;) {
        if (pow_le(m, D, (uint64_t)INT32_MAX - 1, &nc) &&
            (uint64_t)n_min * nc <= (uint64_t)n_eval)
            break;
        if (n_strat_req > 0 || m == 1) return -1;
        --m;
    }
    *n_strat = (int64_t)m;
    *n_cubes = (int64_t)nc;
    *R = n_eval - (int64_t)n_min * (int64_t)nc;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Point in the cube (Alg. 2 getPoint) and bin index i(y) (Eq. 3).             */
/* READING: y = (s + u)/N_st with u = (2r+1)/2^33 from the 32-bit word r, so   */
/* y lies strictly inside (0,1).  With Y = 2(s 2^32 + r) + 1 and P = Y N_g,    */
/* y N_g = P / (N_st 2^33): the bin is its integer part and delta its          */
/* fractional part, both exact; delta is rounded once to double.               */
/* Pinned by exhaustive rational brute force (fractions.Fraction).             */
/* ------------------------------------------------------------------------ */
ORC_EXPORT void orc_point(uint32_t s, uint32_t r, uint32_t n_strat, uint32_t n_g,
                          uint32_t* bin, double* delta)
{
    unsigned __int128 Y = ((unsigned __int128)s << 33) + ((unsigned __int128)r << 1) + 1u;
    unsigned __int128 P = Y * n_g;
    unsigned __int128 den = (unsigned __int128)n_strat << 33;
    unsigned __int128 i = P / den;
    unsigned __int128 rho = P - i * den;
    *bin = (uint32_t)i;
    *delta = (double)(uint64_t)rho / (double)(uint64_t)den;
}

/* ------------------------------------------------------------------------ */
/* Integrand families (Tab. 3 and the benchmark workloads).  Parameter         */
/* layouts (params[]):                                                         */
/*  1 GAUSS_DIAG  A*sum_j exp(-sum_d (x_d-c_j)^2/(2 s^2)); [A, s, M, c_0..]    */
/*  2 GENZ_PPEAK  A*prod_d 1/(a_d^-2 + (x_d-u_d)^2);       [A, a_0.., u_0..]   */
/*  3 GENZ_GAUSS  A*exp(-sum_d a_d^2 (x_d-u_d)^2);          [A, a_0.., u_0..]   */
/*  4 GAUSS_CORR  N(x; mu 1, s^2((1-rho)I + rho 11^T));     [mu, s, rho]        */
/*  5 LINEAR      A*sum_d x_d                               [A]                 */
/*  6 ROOS        A*prod_d |4 x_d - 2|                      [A]                 */
/*  7 CONST       A                                         [A]                 */
/*  8 COSINE      A*prod_d cos x_d                          [A]                 */
/*  9 SIN_EXP     A*(sin x_0 + exp x_1), D >= 2             [A]   (Tab. 3 #1)   */
/* 10 EXP_SQ      A*exp(sum_d x_d^2)                        [A]   (Tab. 3 #4)   */
/* 11 MOROKOFF    A*(1 + 1/D)^D prod_d x_d^(1/D), x >= 0    [A]   (Tab. 3 #6)   */
/* All are written as the formula reads, in FP64 with libm.                    */
/* Pinned by closed-form integrals (erf, arctan, polynomial).                  */
/* ------------------------------------------------------------------------ */
enum { ORC_GAUSS_DIAG = 1, ORC_GENZ_PPEAK = 2, ORC_GENZ_GAUSS = 3,
       ORC_GAUSS_CORR = 4, ORC_LINEAR = 5, ORC_ROOS = 6, ORC_CONST = 7,
       ORC_COSINE = 8, ORC_SIN_EXP = 9, ORC_EXP_SQ = 10, ORC_MOROKOFF = 11 };

ORC_EXPORT double orc_integrand(int family, int D, const double* p, const double* x)
{
    switch (family) {
    case ORC_GAUSS_DIAG: {
        double A = p[0], s = p[1];
        int M = (int)p[2];
        double sum = 0.0;
        for (int j = 0; j < M; ++j) {
            double q = 0.0;
            for (int d = 0; d < D; ++d) {
                double u = x[d] - p[3 + j];
                q += u * u;
            }
            sum += exp(-q / (2.0 * s * s));
        }
        return A * sum;
    }
    case ORC_GENZ_PPEAK: {
        double f = p[0];
        for (int d = 0; d < D; ++d) {
            double a = p[1 + d], u = x[d] - p[1 + D + d];
            f *= 1.0 / (1.0 / (a * a) + u * u);
        }
        return f;
    }
    case ORC_GENZ_GAUSS: {
        double q = 0.0;
        for (int d = 0; d < D; ++d) {
            double a = p[1 + d], u = x[d] - p[1 + D + d];
            q += a * a * u * u;
        }
        return p[0] * exp(-q);
    }
    case ORC_GAUSS_CORR: {
        /* Density of N(mu 1, Sigma), Sigma = s^2 ((1-rho) I + rho 1 1^T).
         * Sigma^-1 = ((I - rho/(1+(D-1)rho) 1 1^T)) / (s^2 (1-rho)) and
         * det Sigma = s^(2D) (1-rho)^(D-1) (1+(D-1)rho). */
        double mu = p[0], s = p[1], rho = p[2];
        double v2 = 0.0, sv = 0.0;
        for (int d = 0; d < D; ++d) {
            double v = x[d] - mu;
            v2 += v * v;
            sv += v;
        }
        double Q = (v2 - rho / (1.0 + (D - 1) * rho) * sv * sv) / (s * s * (1.0 - rho));
        double logdet = 2.0 * D * log(s) + (D - 1) * log(1.0 - rho) + log(1.0 + (D - 1) * rho);
        return exp(-0.5 * Q - 0.5 * D * log(2.0 * M_PI) - 0.5 * logdet);
    }
    case ORC_LINEAR: {
        double s = 0.0;
        for (int d = 0; d < D; ++d) s += x[d];
        return p[0] * s;
    }
    case ORC_ROOS: {
        double f = p[0];
        for (int d = 0; d < D; ++d) f *= fabs(4.0 * x[d] - 2.0);
        return f;
    }
    case ORC_CONST:
        return p[0];
    case ORC_COSINE: {
        double f = p[0];
        for (int d = 0; d < D; ++d) f *= cos(x[d]);
        return f;
    }
    case ORC_SIN_EXP:
        if (D < 2) return NAN;
        return p[0] * (sin(x[0]) + exp(x[1]));
    case ORC_EXP_SQ: {
        double q = 0.0;
        for (int d = 0; d < D; ++d) q += x[d] * x[d];
        return p[0] * exp(q);
    }
    case ORC_MOROKOFF: {
        double f = p[0] * pow(1.0 + 1.0 / D, (double)D);
        for (int d = 0; d < D; ++d) f *= pow(x[d], 1.0 / D);
        return f;
    }
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Allocation of samples to hypercubes (Sec. 2.1.2, Eq. 7; Alg. 1             */
/* updateEvalsPerCube).  n_h ~ sigma_h^beta with sum n_h = N_ev.               */
/* READING: n_min samples are reserved per cube; the rest R is split in        */
/* proportion to q_h = v_h^(beta/2) by exact integer systematic rounding:      */
/*   Q_h = floor(q_h/q_max * 2^32), C_h = Q_0 + .. + Q_h, T = C_{Nc-1},       */
/*   n_h = n_min + floor(R C_h / T) - floor(R C_{h-1} / T).                   */
/* q_max = 0 (or beta = 0) gives Q_h = 1 (uniform split).                      */
/* Pinned by a Python big-integer brute force and invariants.                  */
/* ------------------------------------------------------------------------ */
static double pow_half_beta(double v, double beta)
{   /* v^(beta/2) */
    if (v == 0.0) return 0.0;
    if (beta == 0.75) {           /* v^(3/8) = v^(1/4) * v^(1/8) */
        double a = sqrt(v), b = sqrt(a), c = sqrt(b);
        return b * c;
    }
    if (beta == 1.0) return sqrt(v);
    if (beta == 0.5) return sqrt(sqrt(v));
    if (beta == 2.0) return v;
    return orc_det_exp(0.5 * beta * orc_det_log(v));
}

ORC_EXPORT double orc_alloc_weight(double v, double beta)
{
    return pow_half_beta(v, beta);
}

ORC_EXPORT void orc_alloc(const double* v, int64_t n_cubes, int n_min, int64_t n_eval,
                          double beta, int adapt, uint32_t* nh)
{
    uint64_t R = (uint64_t)(n_eval - (int64_t)n_min * n_cubes);
    uint64_t* Q = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n_cubes);
    double qmax = 0.0;
    if (adapt && beta > 0.0) {
        for (int64_t h = 0; h < n_cubes; ++h) {
            double q = pow_half_beta(v[h], beta);
            if (q > qmax) qmax = q;
        }
    }
    for (int64_t h = 0; h < n_cubes; ++h) {
        if (qmax > 0.0) {
            double q = pow_half_beta(v[h], beta);
            Q[h] = (uint64_t)floor((q / qmax) * 4294967296.0);
        } else {
            Q[h] = 1;
        }
    }
    uint64_t T = 0;
    for (int64_t h = 0; h < n_cubes; ++h) T += Q[h];
    uint64_t Cprev = 0;
    for (int64_t h = 0; h < n_cubes; ++h) {
        uint64_t C = Cprev + Q[h];
        uint64_t hi = (uint64_t)(((unsigned __int128)R * C) / T);
        uint64_t lo = (uint64_t)(((unsigned __int128)R * Cprev) / T);
        nh[h] = (uint32_t)((uint64_t)n_min + hi - lo);
        Cprev = C;
    }
    free(Q);
}

/* ------------------------------------------------------------------------ */
/* Map refinement (Sec. 2.1.1; Alg. 1 adjustWeights + updateMap).              */
/* READING (the paper names the steps -- normalisation, smoothing, damping by  */
/* alpha, aggregation of weights with counts -- without formulas):            */
/*  d_i = H_i/C_i (0 where C_i = 0); smooth with (7,1)/8 at the ends and       */
/*  (1,6,1)/8 inside; normalise e_i = smoothed/S, S summed in bin order;       */
/*  damp g_i = ((1-e_i)/ln(1/e_i))^alpha (0 at e=0, 1 at e=1); rebin so that   */
/*  every new interval holds G/N_g of the damped weight, linearly inside the   */
/*  old interval; the end points stay.  alpha = 0 or all-zero H leaves the     */
/*  axis unchanged.                                                            */
/* Pinned: alpha=0 identity, equal weights keep a uniform grid, tiny grids     */
/* against mpmath, convergence to the inverse CDF of a separable integrand.    */
/* ------------------------------------------------------------------------ */
static double damp(double e, double alpha)
{
    if (e == 0.0) return 0.0;
    if (e == 1.0) return 1.0;
    double t = (1.0 - e) / (-orc_det_log(e));
    if (alpha == 0.5) return sqrt(t);
    if (alpha == 1.0) return t;
    if (alpha == 1.5) return t * sqrt(t);
    return orc_det_exp(alpha * orc_det_log(t));
}

ORC_EXPORT void orc_map_update_axis(double* x /* n_g+1, in/out */, int n_g,
                                    const double* H, const double* C, double alpha)
{
    if (alpha == 0.0) return;
    double* dv = (double*)malloc(sizeof(double) * (size_t)n_g);
    double* e = (double*)malloc(sizeof(double) * (size_t)n_g);
    double* g = (double*)malloc(sizeof(double) * (size_t)n_g);
    double* c = (double*)malloc(sizeof(double) * (size_t)(n_g + 1));
    double* xn = (double*)malloc(sizeof(double) * (size_t)(n_g + 1));
    int any = 0;
    for (int i = 0; i < n_g; ++i) {
        dv[i] = C[i] > 0.0 ? H[i] / C[i] : 0.0;
        if (H[i] != 0.0) any = 1;
    }
    if (!any) goto done;
    if (n_g == 1) {
        e[0] = dv[0];
    } else {
        e[0] = (7.0 * dv[0] + dv[1]) / 8.0;
        for (int i = 1; i < n_g - 1; ++i)
            e[i] = ((dv[i - 1] + 6.0 * dv[i]) + dv[i + 1]) / 8.0;
        e[n_g - 1] = (dv[n_g - 2] + 7.0 * dv[n_g - 1]) / 8.0;
    }
    double S = 0.0;
    for (int i = 0; i < n_g; ++i) S += e[i];
    if (!(S > 0.0)) goto done;
    for (int i = 0; i < n_g; ++i) g[i] = damp(e[i] / S, alpha);
    c[0] = 0.0;
    for (int i = 0; i < n_g; ++i) c[i + 1] = c[i] + g[i];
    double G = c[n_g];
    double dg = G / (double)n_g;
    xn[0] = x[0];
    xn[n_g] = x[n_g];
    int i = 0;
    for (int j = 1; j < n_g; ++j) {
        double tau = (double)j * dg;
        while (!(c[i] <= tau && tau < c[i + 1])) ++i;   /* unique interval */
        double dx = x[i + 1] - x[i];
        xn[j] = fma((tau - c[i]) / g[i], dx, x[i]);
    }
    memcpy(x, xn, sizeof(double) * (size_t)(n_g + 1));
done:
    free(dv); free(e); free(g); free(c); free(xn);
}

/* ------------------------------------------------------------------------ */
/* Combination of iterations (Sec. 2.1.3, Eq. 8-9), chi^2/dof as a            */
/* diagnostic.  READING: an iteration with sigma^2 = 0 is exact; the result is */
/* then the mean of those iterations with sigma^2 = 0.                         */
/* Pinned by hand-computed values.                                             */
/* ------------------------------------------------------------------------ */
ORC_EXPORT void orc_combine(const double* I, const double* s2, int n,
                            double* Ibar, double* s2bar, double* chi2dof)
{
    /* READING: an iteration with sigma_t^2 = 0 is exact (f constant on every
       cube) and decides the result; an "empty" one (I_t = 0 and
       sigma_t^2 = 0: every weight was zero, so the samples missed the
       integrand or it underflowed) says nothing about the variance and is
       left out whenever another iteration has a nonzero estimate. */
    if (n == 0) { *Ibar = 0.0; *s2bar = INFINITY; *chi2dof = 0.0; return; }
    int n_empty = 0;
    for (int t = 0; t < n; ++t)
        if (I[t] == 0.0 && s2[t] == 0.0) ++n_empty;
    if (n_empty == n) { *Ibar = 0.0; *s2bar = 0.0; *chi2dof = 0.0; return; }
    int nz = 0, m = 0;
    double zsum = 0.0;
    for (int t = 0; t < n; ++t) {
        if (I[t] == 0.0 && s2[t] == 0.0) continue;
        ++m;
        if (s2[t] == 0.0) { ++nz; zsum += I[t]; }
    }
    if (nz > 0) {
        *Ibar = zsum / nz;
        *s2bar = 0.0;
        *chi2dof = 0.0;
        return;
    }
    double wsum = 0.0, wisum = 0.0;
    for (int t = 0; t < n; ++t) {
        if (s2[t] == 0.0) continue;
        wsum += 1.0 / s2[t];
        wisum += I[t] / s2[t];
    }
    double Ib = wisum / wsum;
    double chi = 0.0;
    for (int t = 0; t < n; ++t) {
        if (s2[t] == 0.0) continue;
        double u = I[t] - Ib;
        chi += u * u / s2[t];
    }
    *Ibar = Ib;
    *s2bar = 1.0 / wsum;
    *chi2dof = m > 1 ? chi / (m - 1) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* One iteration (Alg. 1 body, Alg. 2 VegasFill) over a given map and         */
/* allocation.  Samples k = 0..N_ev-1 in order; the samples of cube h are the  */
/* contiguous range [start_h, start_h + n_h).  For each sample: the cube's     */
/* digits s_d (dim 0 fastest) give the stratum, the Philox word gives y_d,     */
/* the map gives x_d and J = prod_d N_g dx_d (Eq. 2-3), w = J f(x).            */
/* Per cube (Eq. 5-6): m_h = mean w, v_h = sum (w-m_h)^2/(n_h-1) (two passes,  */
/* READING: the unbiased n-1 form); dI_h = m_h/N_c,                            */
/* var_h = v_h/(N_c^2 n_h); I = sum dI_h, sigma^2 = sum var_h in cube order.   */
/* Per sample and axis: H[d][i_d] += w^2, C[d][i_d] += 1 (READING of          */
/* GetMapWeights).                                                             */
/* ------------------------------------------------------------------------ */
ORC_EXPORT int orc_iterate(
    /* problem */
    int D, int n_g, int64_t n_eval, int64_t n_strat, int64_t n_cubes,
    uint64_t seed, uint32_t inst, uint32_t t, int family, const double* params,
    /* state in */
    const double* grid /* D*(n_g+1) */, const uint32_t* nh /* n_cubes */,
    /* outputs (any may be NULL) */
    double* m_out /* n_cubes */, double* v_out /* n_cubes */,
    double* H /* D*n_g */, double* C /* D*n_g */,
    double* I_out, double* s2_out, int64_t* n_nonfinite)
{
    double* w = NULL;
    uint32_t maxn = 0;
    int64_t total = 0;
    for (int64_t h = 0; h < n_cubes; ++h) {
        if (nh[h] > maxn) maxn = nh[h];
        if (nh[h] < 2) return -2;          /* v_h needs two samples */
        total += nh[h];
    }
    if (total != n_eval) return -2;        /* the allocation spends N_ev exactly */
    w = (double*)malloc(sizeof(double) * (size_t)(maxn ? maxn : 1));
    if (!w) return -1;
    if (H) memset(H, 0, sizeof(double) * (size_t)D * n_g);
    if (C) memset(C, 0, sizeof(double) * (size_t)D * n_g);
    uint32_t* s = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)D);
    uint32_t* bins = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)D);
    double* x = (double*)malloc(sizeof(double) * (size_t)D);
    double Nc = (double)n_cubes;
    double Nc2 = Nc * Nc;
    double I = 0.0, S2 = 0.0;
    int64_t nonfinite = 0;
    uint64_t k = 0;
    for (int64_t h = 0; h < n_cubes; ++h) {
        /* stratum digits of h, dimension 0 fastest */
        int64_t rem = h;
        for (int d = 0; d < D; ++d) { s[d] = (uint32_t)(rem % n_strat); rem /= n_strat; }
        uint32_t n = nh[h];
        for (uint32_t j = 0; j < n; ++j, ++k) {
            double J = 1.0;
            for (int d = 0; d < D; ++d) {
                uint32_t r = orc_word(seed, inst, t, k, d);
                double delta;
                orc_point(s[d], r, (uint32_t)n_strat, (uint32_t)n_g, &bins[d], &delta);
                const double* g = grid + (size_t)d * (n_g + 1);
                double dx = g[bins[d] + 1] - g[bins[d]];
                x[d] = fma(dx, delta, g[bins[d]]);
                J = J * ((double)n_g * dx);
            }
            double f = orc_integrand(family, D, params, x);
            double wk = J * f;
            if (!isfinite(wk)) { ++nonfinite; wk = 0.0; }
            w[j] = wk;
            for (int d = 0; d < D; ++d) {
                if (H) H[(size_t)d * n_g + bins[d]] += wk * wk;
                if (C) C[(size_t)d * n_g + bins[d]] += 1.0;
            }
        }
        double sum = 0.0;
        for (uint32_t j = 0; j < n; ++j) sum += w[j];
        double m = sum / (double)n;
        double ss = 0.0;
        for (uint32_t j = 0; j < n; ++j) { double u = w[j] - m; ss += u * u; }
        double v = ss / (double)(n - 1);
        if (m_out) m_out[h] = m;
        if (v_out) v_out[h] = v;
        I += m / Nc;
        S2 += v / (Nc2 * (double)n);
    }
    if (I_out) *I_out = I;
    if (s2_out) *s2_out = S2;
    if (n_nonfinite) *n_nonfinite = nonfinite;
    free(w); free(s); free(bins); free(x);
    return 0;
}

/* One sample's intermediate values, for detailed checks. */
ORC_EXPORT void orc_sample(int D, int n_g, int64_t n_strat, uint64_t seed, uint32_t inst,
                           uint32_t t, uint64_t k, int64_t h, const double* grid,
                           int family, const double* params,
                           uint32_t* bins, double* delta, double* x, double* J, double* f)
{
    int64_t rem = h;
    double Jv = 1.0;
    for (int d = 0; d < D; ++d) {
        uint32_t sd = (uint32_t)(rem % n_strat);
        rem /= n_strat;
        uint32_t r = orc_word(seed, inst, t, k, d);
        orc_point(sd, r, (uint32_t)n_strat, (uint32_t)n_g, &bins[d], &delta[d]);
        const double* g = grid + (size_t)d * (n_g + 1);
        double dx = g[bins[d] + 1] - g[bins[d]];
        x[d] = fma(dx, delta[d], g[bins[d]]);
        Jv = Jv * ((double)n_g * dx);
    }
    *J = Jv;
    *f = orc_integrand(family, D, params, x);
}

/* Initial map (READING: uniform): x_{d,i} = a_d + ((b_d - a_d) i)/N_g. */
ORC_EXPORT void orc_init_grid(int D, int n_g, const double* lo, const double* hi, double* grid)
{
    for (int d = 0; d < D; ++d)
        for (int i = 0; i <= n_g; ++i)
            grid[(size_t)d * (n_g + 1) + i] = lo[d] + ((hi[d] - lo[d]) * (double)i) / (double)n_g;
}

/* ------------------------------------------------------------------------ */
/* Whole run (Alg. 1): n_adapt iterations whose estimates are discarded        */
/* (the paper's skip), then n_iter iterations combined by Eq. 8-9.  After      */
/* every iteration the allocation (beta) and the map (alpha) are updated,      */
/* READING: also after the last one, so that the state can be continued.      */
/* The allocation update uses the v_h of the samples just drawn; the map the   */
/* histograms of the same samples.                                             */
/* ------------------------------------------------------------------------ */
ORC_EXPORT int orc_run(int D, int n_g, int64_t n_eval, int n_min, int n_strat_req,
                       double alpha, double beta, uint64_t seed, uint32_t inst,
                       int adapt_map, int adapt_strat, int family, const double* params,
                       const double* lo, const double* hi, int n_adapt, int n_iter,
                       double* grid_io /* D*(n_g+1) or NULL: uniform start */,
                       uint32_t* nh_io /* n_cubes or NULL: uniform start */,
                       uint32_t t0,
                       double* I_t /* n_adapt+n_iter */, double* s2_t,
                       double* result /* [Ibar, s2bar, chi2dof] */,
                       int64_t* n_nonfinite)
{
    int64_t ns, nc, R;
    if (orc_strata(n_eval, D, n_min, n_strat_req, &ns, &nc, &R) != 0) return -1;
    double* grid = (double*)malloc(sizeof(double) * (size_t)D * (n_g + 1));
    uint32_t* nh = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nc);
    double* v = (double*)malloc(sizeof(double) * (size_t)nc);
    double* H = (double*)malloc(sizeof(double) * (size_t)D * n_g);
    double* C = (double*)malloc(sizeof(double) * (size_t)D * n_g);
    if (grid_io) memcpy(grid, grid_io, sizeof(double) * (size_t)D * (n_g + 1));
    else orc_init_grid(D, n_g, lo, hi, grid);
    if (nh_io) memcpy(nh, nh_io, sizeof(uint32_t) * (size_t)nc);
    else orc_alloc(v, nc, n_min, n_eval, beta, 0, nh);
    int64_t nnf = 0;
    int total = n_adapt + n_iter;
    for (int it = 0; it < total; ++it) {
        double I, s2;
        int64_t bad = 0;
        orc_iterate(D, n_g, n_eval, ns, nc, seed, inst, t0 + (uint32_t)it, family, params,
                    grid, nh, NULL, v, H, C, &I, &s2, &bad);
        nnf += bad;
        I_t[it] = I;
        s2_t[it] = s2;
        orc_alloc(v, nc, n_min, n_eval, beta, adapt_strat, nh);
        if (adapt_map)
            for (int d = 0; d < D; ++d)
                orc_map_update_axis(grid + (size_t)d * (n_g + 1), n_g,
                                    H + (size_t)d * n_g, C + (size_t)d * n_g, alpha);
    }
    orc_combine(I_t + n_adapt, s2_t + n_adapt, n_iter, &result[0], &result[1], &result[2]);
    if (grid_io) memcpy(grid_io, grid, sizeof(double) * (size_t)D * (n_g + 1));
    if (nh_io) memcpy(nh_io, nh, sizeof(uint32_t) * (size_t)nc);
    if (n_nonfinite) *n_nonfinite = nnf;
    free(grid); free(nh); free(v); free(H); free(C);
    return 0;
}
