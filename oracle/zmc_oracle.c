/*
 * zmc_oracle.c -- CPU oracle for the stratified-sampling + heuristic-tree-search
 * Monte Carlo integrator of "ZMCintegral: a Package for Multi-Dimensional Monte
 * Carlo Integration on Multi-GPUs" (Wu, Zhang, Pang, Wang; arXiv:1902.07916).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU product path
 * neither includes, links nor calls anything here, and this file includes
 * nothing from the product path.
 *
 * Plain, single-threaded, FP64, libm.  Every step follows the method's
 * description in the paper's Sec. 2.1 in the order the paper gives it; the
 * points the paper leaves open are fixed by the readings listed in the header
 * comment of each function.  No blocking, fusion or reordering: sums run
 * serially in list / sample order.
 *
 * Parity status per function:
 *   oracle_philox4x32_10  pinned: published known-answer vectors + rocRAND.
 *   oracle_uniform        pinned: exact special cases, dyadic grid, KS test.
 *   oracle_cube_bounds    pinned: children tile the parent; leaves tile the domain.
 *   oracle_cube_trial     pinned: closed forms (erf, complex exponential, atan,
 *                         inclusion-exclusion, monomials), 2-D Riemann sums.
 *   oracle_threshold      pinned: numpy population std; hand examples; values
 *                         whose squared deviations underflow (numpy on
 *                         values scaled by a power of two).
 *   oracle_set_user       pinned: a user function equal to a registry
 *                         integrand reproduces it bit for bit; closed form.
 *   oracle_integrate      pinned: closed forms within k*stderr, constant
 *                         integrand exact, Cantelli bound on selections,
 *                         paper's printed anchors (Tables 1, 2) as loose sanity.
 *   sum_abs / per-cube sa pinned: equal to +-integral where f keeps one sign
 *                         (refined, truncated and rtol-stopped trees), the
 *                         closed forms of the integral of |sin| (1-D) and
 *                         |sin(x + y)| (2-D) where it changes sign.
 *   the exact tree of the large 6-D / 9-D workloads has no external value of
 *   its own: it is the composition of the steps pinned above (per-cube
 *   estimates, threshold, strict selection, children), each pinned at sizes
 *   where an independent value exists.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_DIM 16
#define OR_MAX_LEVELS 16
#define OR_MAX_PARAMS (2 * OR_MAX_DIM + 2)

enum {
    OR_GAUSS = 0,
    OR_SIN_SUM = 1,
    OR_GENZ_OSC = 2,
    OR_GENZ_PPEAK = 3,
    OR_GENZ_CPEAK = 4,
    OR_GENZ_GAUSS = 5,
    OR_CONST = 6,
    OR_MONOMIAL = 7,
    OR_N_INTEGRANDS = 8
};

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENONFINITE = -3, OR_ENOMEM = -2 };
enum { OR_F_TRUNCATED = 1, OR_F_RTOL_MET = 2 };

typedef struct {
    int32_t integrand;
    int32_t dim;
    int32_t divisions;   /* root sub-domains per axis: k = divisions^dim   */
    int32_t trials;      /* n1: independent repetitions per sub-domain     */
    int32_t max_depth;   /* refinement rounds after the root division      */
    int32_t n_params;
    int32_t split;       /* b: a split cuts every axis into b parts (b^D
                            children); 2 = bisection (default reading), b = d
                            = the paper's split into k equal parts      */
    int32_t scope;       /* threshold population: 0 = all cubes of a level
                            (default reading), 1 = the children of one
                            parent (roots: all roots)                       */
    int64_t samples;     /* N: points per trial per sub-domain             */
    int64_t max_cubes_per_level;
    double sigma_mult;
    double rtol;         /* 0 = off */
    uint64_t seed;
    double lower[OR_MAX_DIM];
    double upper[OR_MAX_DIM];
    double params[OR_MAX_PARAMS];
} oracle_problem;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As    */
/* Easy as 1, 2, 3", SC'11, Sec. 3.2 / Table 2): ten rounds of two 32x32->64  */
/* multiplies by the constants 0xD2511F53 and 0xCD9E8D57, an S-box that       */
/* swaps the products' halves into the other lanes XORed with the key, and a  */
/* Weyl key schedule with increments 0x9E3779B9 and 0xBB67AE85.               */
/* ------------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

/* Uniform deviate from one 32-bit word: the top 23 bits select one of 2^23
 * equal cells of (0,1) and u is that cell's midpoint, (2*(w>>9)+1) * 2^-24.
 * Exact in FP32 and FP64, never 0 or 1.  (The paper's produce-at-calculation
 * scheme, Sec. 2.2, fixes no generator or mapping; this is the reading used.) */
double oracle_uniform(uint32_t w)
{
    uint32_t cell = w >> 9;
    return (double)(2u * cell + 1u) * 0x1p-24;
}

/* Cube ids hold up to 84 bits: the low 64 in uid, bits 64..83 in uid_hi. */
typedef unsigned __int128 or_u128;
#define OR_ID_BITS 84

static or_u128 wide_id(uint64_t lo, uint32_t hi) { return ((or_u128)hi << 64) | (or_u128)lo; }

/* Counter word 1 of the stream of trial t of the cube (uid, level): bits 0..7
 * the trial, 8..11 the level, 12..31 the id bits above 64 (zero for every id
 * below 2^64, whose streams are therefore those of 64-bit ids). */
static uint32_t ctr_word1(int trial, int level, uint32_t uid_hi)
{
    return (uint32_t)trial | ((uint32_t)level << 8) | (uid_hi << 12);
}

/* The RNG word that drives dimension i of sample s in trial t of the cube
 * (uid, level): word n = s*D + i of the stream keyed by the 64-bit seed, with
 * counter (n >> 2, t | level << 8 | uid_hi << 12, lo32(uid), hi32(uid)), lane
 * n & 3. */
uint32_t oracle_word_w(uint64_t seed, uint64_t uid, uint32_t uid_hi, int level, int trial, int dim, int64_t s,
                       int i)
{
    uint64_t n = (uint64_t)s * (uint64_t)dim + (uint64_t)i;
    uint32_t ctr[4] = {(uint32_t)(n >> 2), ctr_word1(trial, level, uid_hi), (uint32_t)uid, (uint32_t)(uid >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[n & 3u];
}

uint32_t oracle_word(uint64_t seed, uint64_t uid, int level, int trial, int dim, int64_t s, int i)
{
    return oracle_word_w(seed, uid, 0, level, trial, dim, s, i);
}

/* ------------------------------------------------------------------------- */
/* Sub-domain geometry (Sec. 2.1: the domain is divided into k equal          */
/* hypercubes; a sub-domain that must be recalculated is split again).        */
/* Reading: k = d^D root cubes numbered r = 0..d^D-1 in row-major order with   */
/* axis 0 most significant; a split bisects every axis (2^D children), child  */
/* c of parent uid gets uid' = (uid << D) | c and bit (D-1-i) of c is the      */
/* upper/lower half along axis i.                                              */
/* ------------------------------------------------------------------------- */

static uint64_t ipow_u64(uint64_t b, int e)
{
    uint64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

/* Integer lattice coordinates of a cube at `level`: cell index along each
 * axis on a grid of d * b^level cells.  uid = root * (b^D)^level + path,
 * the path holding one base-b^D digit per split, and each digit c holding
 * the part along axis i as its base-b digit D-1-i (axis 0 most significant).
 * For b = 2 this is uid' = (uid << D) | c with bit D-1-i of c for axis i. */
void oracle_cube_lattice_w(int dim, int divisions, int split, int level, uint64_t uid_lo, uint32_t uid_hi,
                           uint64_t* K)
{
    const or_u128 uid = wide_id(uid_lo, uid_hi);
    const or_u128 kids = (or_u128)ipow_u64((uint64_t)split, dim);
    or_u128 path_scale = 1; /* (b^D)^level; saturates once it exceeds every id */
    int full = 0;
    for (int j = 0; j < level; ++j) {
        if (path_scale > ((or_u128)1 << OR_ID_BITS) / kids) full = 1;
        else path_scale *= kids;
    }
    /* the root index sits above the path digits (none left when they fill the id) */
    or_u128 root = full ? 0 : uid / path_scale;
    for (int i = dim - 1; i >= 0; --i) {
        K[i] = (uint64_t)(root % (or_u128)divisions);
        root /= (or_u128)divisions;
    }
    for (int j = 1; j <= level; ++j) {
        or_u128 c = uid;
        for (int t = 0; t < level - j; ++t) c /= kids;
        c %= kids;
        for (int i = 0; i < dim; ++i) {
            or_u128 digit = c;
            for (int t = 0; t < dim - 1 - i; ++t) digit /= (or_u128)split;
            K[i] = (uint64_t)split * K[i] + (uint64_t)(digit % (or_u128)split);
        }
    }
}

void oracle_cube_lattice(int dim, int divisions, int split, int level, uint64_t uid, uint64_t* K)
{
    oracle_cube_lattice_w(dim, divisions, split, level, uid, 0, K);
}

/* Lower corner, edge lengths and volume of the cube (uid, level). */
void oracle_cube_bounds_w(const oracle_problem* p, int level, uint64_t uid, uint32_t uid_hi, double* lo, double* h,
                          double* vol)
{
    uint64_t K[OR_MAX_DIM];
    oracle_cube_lattice_w(p->dim, p->divisions, p->split, level, uid, uid_hi, K);
    const double parts = (double)ipow_u64((uint64_t)p->split, level); /* b^level, exact */
    double v = 1.0;
    for (int i = 0; i < p->dim; ++i) {
        double h0 = (p->upper[i] - p->lower[i]) / (double)p->divisions;
        h[i] = h0 / parts;
        lo[i] = fma((double)K[i], h[i], p->lower[i]);
        v = v * h[i];
    }
    *vol = v;
}

void oracle_cube_bounds(const oracle_problem* p, int level, uint64_t uid, double* lo, double* h, double* vol)
{
    oracle_cube_bounds_w(p, level, uid, 0, lo, h, vol);
}

/* ------------------------------------------------------------------------- */
/* Integrands.  Sec. 3 defines f1 = sin(sum x_i) and the normalised 9-D       */
/* Gaussian f2; the Genz families and the test-only constant / monomial are   */
/* the registry the workloads draw from.                                       */
/* ------------------------------------------------------------------------- */
/* User-defined integrands (the paper's package takes general user
 * functions, abstract and Sec. 3.3): ids 100.. call a registered function
 * f(x, params, D). */
#define OR_USER_BASE 100
#define OR_MAX_USER 64
typedef double (*oracle_user_fn)(const double* x, const double* p, int dim);
static oracle_user_fn g_user_fn[OR_MAX_USER];
static int g_user_np[OR_MAX_USER];

int oracle_set_user(int id, oracle_user_fn f, int n_params)
{
    if (id < OR_USER_BASE || id >= OR_USER_BASE + OR_MAX_USER || !f || n_params < 0 || n_params > OR_MAX_PARAMS)
        return OR_EINVAL;
    g_user_fn[id - OR_USER_BASE] = f;
    g_user_np[id - OR_USER_BASE] = n_params;
    return OR_OK;
}

static int is_user(int id)
{
    return id >= OR_USER_BASE && id < OR_USER_BASE + OR_MAX_USER && g_user_fn[id - OR_USER_BASE] != NULL;
}

int oracle_n_params(int id, int dim)
{
    if (is_user(id)) return g_user_np[id - OR_USER_BASE];
    switch (id) {
    case OR_GAUSS: return 2 + dim;
    case OR_SIN_SUM: return 0;
    case OR_GENZ_OSC: return 1 + dim;
    case OR_GENZ_PPEAK: return 2 * dim;
    case OR_GENZ_CPEAK: return dim;
    case OR_GENZ_GAUSS: return 2 * dim;
    case OR_CONST: return 1;
    case OR_MONOMIAL: return dim;
    default: return -1;
    }
}

double oracle_f(int id, const double* prm, int dim, const double* x)
{
    const double two_pi = 6.283185307179586476925286766559;
    if (is_user(id)) return g_user_fn[id - OR_USER_BASE](x, prm, dim);
    switch (id) {
    case OR_GAUSS: { /* A * exp(-sum (x_i - mu_i)^2 / (2 sigma^2)) */
        double sigma = prm[0], A = prm[1], q = 0.0;
        for (int i = 0; i < dim; ++i) {
            double d = x[i] - prm[2 + i];
            q += d * d;
        }
        return A * exp(-q / (2.0 * sigma * sigma));
    }
    case OR_SIN_SUM: { /* sin(sum x_i) */
        double t = 0.0;
        for (int i = 0; i < dim; ++i) t += x[i];
        return sin(t);
    }
    case OR_GENZ_OSC: { /* cos(2 pi u + sum c_i x_i) */
        double t = two_pi * prm[0];
        for (int i = 0; i < dim; ++i) t += prm[1 + i] * x[i];
        return cos(t);
    }
    case OR_GENZ_PPEAK: { /* prod 1 / (c_i^-2 + (x_i - w_i)^2) */
        double f = 1.0;
        for (int i = 0; i < dim; ++i) {
            double c = prm[i], d = x[i] - prm[dim + i];
            f *= 1.0 / (1.0 / (c * c) + d * d);
        }
        return f;
    }
    case OR_GENZ_CPEAK: { /* (1 + sum c_i x_i)^-(D+1) */
        double t = 1.0;
        for (int i = 0; i < dim; ++i) t += prm[i] * x[i];
        return pow(t, -(double)(dim + 1));
    }
    case OR_GENZ_GAUSS: { /* exp(-sum c_i^2 (x_i - w_i)^2) */
        double q = 0.0;
        for (int i = 0; i < dim; ++i) {
            double c = prm[i], d = x[i] - prm[dim + i];
            q += c * c * d * d;
        }
        return exp(-q);
    }
    case OR_CONST:
        return prm[0];
    case OR_MONOMIAL: { /* prod x_i^p_i, integer p_i in 0..16 */
        double f = 1.0;
        for (int i = 0; i < dim; ++i) f *= pow(x[i], prm[i]);
        return f;
    }
    default:
        return NAN;
    }
}

/* Sample point s of trial t in cube (uid, level): x_i = fma(h_i, u, lo_i). */
void oracle_sample_x_w(const oracle_problem* p, int level, uint64_t uid, uint32_t uid_hi, int trial, int64_t s,
                       double* x)
{
    double lo[OR_MAX_DIM], h[OR_MAX_DIM], vol;
    oracle_cube_bounds_w(p, level, uid, uid_hi, lo, h, &vol);
    for (int i = 0; i < p->dim; ++i) {
        double u = oracle_uniform(oracle_word_w(p->seed, uid, uid_hi, level, trial, p->dim, s, i));
        x[i] = fma(h[i], u, lo[i]);
    }
}

void oracle_sample_x(const oracle_problem* p, int level, uint64_t uid, int trial, int64_t s, double* x)
{
    oracle_sample_x_w(p, level, uid, 0, trial, s, x);
}

/* ------------------------------------------------------------------------- */
/* One direct Monte Carlo estimate of the integral over one sub-domain         */
/* (Sec. 2.1: each hypercube's integral is a plain direct Monte Carlo       */
/* estimate): I_t = V * (1/N) sum_s f(x_s).  Diagnostics S2 = sum             */
/* f^2 and SA = sum |f| never feed a decision.  Returns 0, or OR_ENONFINITE   */
/* if any f was not finite.                                                    */
/* ------------------------------------------------------------------------- */
int oracle_cube_trial_w(const oracle_problem* p, int level, uint64_t uid, uint32_t uid_hi, int trial, double* I_t,
                        double* S1_out, double* S2_out, double* SA_out)
{
    const int D = p->dim;
    double lo[OR_MAX_DIM], h[OR_MAX_DIM], vol, x[OR_MAX_DIM];
    oracle_cube_bounds_w(p, level, uid, uid_hi, lo, h, &vol);
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    uint32_t block[4];
    uint64_t cached = ~0ull;
    double S1 = 0.0, S2 = 0.0, SA = 0.0;
    int finite = 1;
    for (int64_t s = 0; s < p->samples; ++s) {
        for (int i = 0; i < D; ++i) {
            uint64_t n = (uint64_t)s * (uint64_t)D + (uint64_t)i;
            if ((n >> 2) != cached) { /* one Philox block serves four words */
                cached = n >> 2;
                uint32_t ctr[4] = {(uint32_t)cached, ctr_word1(trial, level, uid_hi), (uint32_t)uid,
                                   (uint32_t)(uid >> 32)};
                oracle_philox4x32_10(ctr, key, block);
            }
            double u = oracle_uniform(block[n & 3u]);
            x[i] = fma(h[i], u, lo[i]);
        }
        double f = oracle_f(p->integrand, p->params, D, x);
        if (!isfinite(f)) finite = 0;
        S1 += f;
        S2 += f * f;
        SA += fabs(f);
    }
    if (S1_out) *S1_out = S1;
    if (S2_out) *S2_out = S2;
    if (SA_out) *SA_out = SA;
    *I_t = vol * (S1 / (double)p->samples);
    return finite ? OR_OK : OR_ENONFINITE;
}

int oracle_cube_trial(const oracle_problem* p, int level, uint64_t uid, int trial, double* I_t, double* S1_out,
                      double* S2_out, double* SA_out)
{
    return oracle_cube_trial_w(p, level, uid, 0, trial, I_t, S1_out, S2_out, SA_out);
}

/* Population standard deviation of x[0..n) around mean (Sec. 2.1 uses the
 * standard deviation of the trial values and of the cubes' deviations):
 * sqrt(sum (x - mean)^2 / n), serial sum.  Reading: each deviation is scaled
 * by 2^-e, e the binary exponent of the largest |x - mean| (frexp), before
 * it is squared, and the root by 2^e after.  Powers of two scale exactly, so
 * wherever the unscaled squares neither underflow nor overflow this is the
 * same number bit for bit; where they would (deviations below ~1e-154, as in
 * the tails of a narrow Gaussian), the deviations are not lost. */
static double or_pop_std(const double* x, int64_t n, double mean)
{
    double dmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double d = fabs(x[i] - mean);
        if (d > dmax) dmax = d;
    }
    int e = 0;
    if (isfinite(dmax) && dmax > 0.0) (void)frexp(dmax, &e);
    double ss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double d = ldexp(x[i] - mean, -e);
        ss += d * d;
    }
    return ldexp(sqrt(ss / (double)n), e);
}

/* Mean and standard deviation of the n1 trial values of one sub-domain
 * (Sec. 2.1).  Reading: population std (ddof = 0, or_pop_std), two passes,
 * serial sums.  I_out (length n1) may be NULL. */
int oracle_cube_w(const oracle_problem* p, int level, uint64_t uid, uint32_t uid_hi, double* I_out, double* m_out,
                  double* s_out, double* SA_out)
{
    const int n1 = p->trials;
    double I[256];
    double sa_tot = 0.0;
    int st = OR_OK;
    for (int t = 0; t < n1; ++t) {
        double sa;
        if (oracle_cube_trial_w(p, level, uid, uid_hi, t, &I[t], NULL, NULL, &sa) != OR_OK) st = OR_ENONFINITE;
        sa_tot += sa;
        if (I_out) I_out[t] = I[t];
    }
    double sum = 0.0;
    for (int t = 0; t < n1; ++t) sum += I[t];
    double m = sum / (double)n1;
    *m_out = m;
    *s_out = or_pop_std(I, n1, m);
    if (SA_out) {
        double lo[OR_MAX_DIM], h[OR_MAX_DIM], vol;
        oracle_cube_bounds_w(p, level, uid, uid_hi, lo, h, &vol);
        *SA_out = vol * (sa_tot / ((double)p->samples * (double)n1));
    }
    if (!isfinite(*m_out) || !isfinite(*s_out)) st = OR_ENONFINITE;
    return st;
}

int oracle_cube(const oracle_problem* p, int level, uint64_t uid, double* I_out, double* m_out, double* s_out,
                double* SA_out)
{
    return oracle_cube_w(p, level, uid, 0, I_out, m_out, s_out, SA_out);
}

/* Threshold over one level's standard deviations (Sec. 2.1: the threshold is
 * set from the mean and the standard deviation of the k standard deviations;
 * Sec. 3 applies it as a five-sigma cut).  Reading: thr = mean(s) +
 * sigma_mult * std(s), population std (or_pop_std), two passes, serial
 * sums. */
double oracle_threshold(const double* s, int64_t n, double sigma_mult, double* mu_out, double* sd_out)
{
    double sum = 0.0;
    for (int64_t c = 0; c < n; ++c) sum += s[c];
    double mu = sum / (double)n;
    double sd = or_pop_std(s, n, mu);
    if (mu_out) *mu_out = mu;
    if (sd_out) *sd_out = sd;
    return mu + sigma_mult * sd;
}

/* The b^D children of a cube, in order c = 0 .. b^D - 1: uid * b^D + c. */
void oracle_children_w(uint64_t uid, uint32_t uid_hi, int dim, int split, uint64_t* out, uint32_t* out_hi)
{
    uint64_t nc = ipow_u64((uint64_t)split, dim);
    for (uint64_t c = 0; c < nc; ++c) {
        or_u128 k = wide_id(uid, uid_hi) * (or_u128)nc + (or_u128)c;
        out[c] = (uint64_t)k;
        if (out_hi) out_hi[c] = (uint32_t)(k >> 64);
    }
}

void oracle_children(uint64_t uid, int dim, int split, uint64_t* out)
{
    oracle_children_w(uid, 0, dim, split, out, NULL);
}

/* ------------------------------------------------------------------------- */
/* Argument checks shared by every entry point of the oracle.                  */
/* ------------------------------------------------------------------------- */
int oracle_validate(const oracle_problem* p)
{
    if (p->dim < 1 || p->dim > OR_MAX_DIM) return OR_EINVAL;
    if (!is_user(p->integrand) && (p->integrand < 0 || p->integrand >= OR_N_INTEGRANDS)) return OR_EINVAL;
    if (p->n_params != oracle_n_params(p->integrand, p->dim)) return OR_EINVAL;
    /* parameter values are not checked: an integrand that evaluates to a
     * non-finite value fails the run with OR_ENONFINITE instead */
    if (p->integrand == OR_MONOMIAL)
        for (int j = 0; j < p->n_params; ++j)
            if (!(p->params[j] >= 0.0 && p->params[j] <= 16.0 && p->params[j] == floor(p->params[j])))
                return OR_EINVAL;
    if (p->divisions < 1) return OR_EINVAL;
    if (p->split < 2 || p->split > 64) return OR_EINVAL;
    if (p->scope != 0 && p->scope != 1) return OR_EINVAL;
    {
        /* at most 2^24 children per split */
        uint64_t kids = 1;
        for (int i = 0; i < p->dim; ++i) {
            kids *= (uint64_t)p->split;
            if (kids > (1ull << 24)) return OR_EINVAL;
        }
    }
    if (p->samples < 1) return OR_EINVAL;
    if ((uint64_t)p->samples * (uint64_t)p->dim > (1ull << 34)) return OR_EINVAL;
    if (p->trials < 2 || p->trials > 255) return OR_EINVAL;
    if (p->max_depth < 0 || p->max_depth >= OR_MAX_LEVELS) return OR_EINVAL;
    if (!isfinite(p->sigma_mult) || p->sigma_mult < 0.0) return OR_EINVAL;
    if (!isfinite(p->rtol) || p->rtol < 0.0) return OR_EINVAL;
    if (p->max_cubes_per_level < 1) return OR_EINVAL;
    for (int i = 0; i < p->dim; ++i)
        if (!isfinite(p->lower[i]) || !isfinite(p->upper[i]) || !(p->lower[i] < p->upper[i])) return OR_EINVAL;
    /* every id below d^D * (b^D)^max_depth must fit OR_ID_BITS bits (for
     * b = 2: the root bits plus D bits per refinement); d^D itself must fit
     * 64 bits, and so must the lattice cells per axis, d * b^max_depth */
    {
        const or_u128 lim = (or_u128)1 << OR_ID_BITS;
        or_u128 top = 1, cells = (or_u128)p->divisions;
        for (int i = 0; i < p->dim; ++i) {
            top *= (or_u128)p->divisions;
            if (top > (or_u128)(~0ull)) return OR_EINVAL;
        }
        for (int l = 0; l < p->max_depth; ++l) {
            for (int i = 0; i < p->dim; ++i) {
                top *= (or_u128)p->split;
                if (top > lim) return OR_EINVAL;
            }
            cells *= (or_u128)p->split;
            if (cells > ((or_u128)1 << 64)) return OR_EINVAL;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* The whole heuristic tree search (Sec. 2.1).                                 */
/*                                                                             */
/* Readings of points the paper leaves open:                                   */
/*  - level 0 holds the k = d^D root cubes; max_depth counts refinement rounds */
/*    (cube ids hold up to 84 bits: see oracle_word_w);                       */
/*    after it, so the paper's "partition depth" is max_depth + 1;             */
/*  - a selected cube is split into 2^D children (every axis bisected; with  */
/*    split = b, b^D children, b = d being the paper's k equal parts        */
/*    sub-sub-domains"), and the children replace it (its own mean and std  */
/*    are dropped);                                                          */
/*  - the threshold is recomputed over each new list of sub-domains, i.e. per */
/*    level over all of that level's cubes (scope 1: over the children of   */
/*    each parent);                                                          */
/*  - selection is the strict "s > thr"; at level max_depth every cube is      */
/*    accepted;                                                                */
/*  - result = sum of accepted means; std = sqrt(sum of accepted s^2);         */
/*    stderr = sqrt(sum s^2 / (n1 - 1));                                       */
/*  - if the next list would exceed max_cubes_per_level, the selected cubes    */
/*    are accepted instead and the search stops (flag TRUNCATED);              */
/*  - with rtol > 0, after each level the running estimate (accepted so far   */
/*    plus the cubes that would be split) is formed and the search stops once */
/*    its stderr <= rtol * |estimate| (flag RTOL_MET).                         */
/*                                                                             */
/* Replay (for comparing against a run whose rounding differs): when a cube's */
/* std lies within band_eps * thr of the threshold and the replay list holds  */
/* its uid for this level, the replayed decision is adopted.                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    uint64_t* uid;       /* id bits 0..63 */
    uint32_t* uid_hi;    /* id bits 64..83 */
    double* m;
    double* s;
    double* I;      /* n * trials */
    double* sa;     /* per-cube estimate of the integral of |f| */
    uint8_t* sel;
    double thr, mu, sd, min_margin;
    int64_t n_sel;
    int64_t n_in_band;
    int64_t n_replayed;
} oracle_level;

typedef struct {
    int status;
    int flags;
    int levels_run;
    double integral;
    double std;
    double stderr_;
    double sum_abs; /* estimate of the integral of |f| over the domain */
    uint64_t n_samples;
    uint64_t n_cubes;
    oracle_level level[OR_MAX_LEVELS];
} oracle_run;

typedef struct {
    int32_t n_levels;
    int64_t n[OR_MAX_LEVELS];
    const uint64_t* uid[OR_MAX_LEVELS];    /* ascending by (uid_hi, uid) */
    const uint32_t* uid_hi[OR_MAX_LEVELS]; /* NULL: all zero */
    const uint8_t* sel[OR_MAX_LEVELS];
} oracle_replay;

static or_u128 replay_id(const oracle_replay* rp, int level, int64_t i)
{
    return wide_id(rp->uid[level][i], rp->uid_hi[level] ? rp->uid_hi[level][i] : 0u);
}

static int replay_lookup(const oracle_replay* rp, int level, or_u128 uid, int* decision)
{
    if (!rp || level >= rp->n_levels || !rp->uid[level]) return 0;
    int64_t a = 0, b = rp->n[level];
    while (a < b) {
        int64_t mid = a + (b - a) / 2;
        if (replay_id(rp, level, mid) < uid) a = mid + 1;
        else b = mid;
    }
    if (a < rp->n[level] && replay_id(rp, level, a) == uid) {
        *decision = rp->sel[level][a] ? 1 : 0;
        return 1;
    }
    return 0;
}

void oracle_free(oracle_run* r)
{
    if (!r) return;
    for (int l = 0; l < OR_MAX_LEVELS; ++l) {
        free(r->level[l].uid);
        free(r->level[l].uid_hi);
        free(r->level[l].m);
        free(r->level[l].s);
        free(r->level[l].I);
        free(r->level[l].sa);
        free(r->level[l].sel);
    }
    free(r);
}

oracle_run* oracle_integrate(const oracle_problem* p, const oracle_replay* rp, double band_eps)
{
    oracle_run* r = (oracle_run*)calloc(1, sizeof(oracle_run));
    if (!r) return NULL;
    r->status = oracle_validate(p);
    if (r->status != OR_OK) return r;

    const int D = p->dim, n1 = p->trials;
    uint64_t k = 1;
    for (int i = 0; i < D; ++i) k *= (uint64_t)p->divisions;
    if (k > (uint64_t)p->max_cubes_per_level) {
        r->status = OR_EINVAL;
        return r;
    }

    /* level 0: every root cube, ascending */
    int64_t n = (int64_t)k;
    uint64_t* list = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    uint32_t* list_hi = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    if (!list || !list_hi) { free(list); free(list_hi); r->status = OR_ENOMEM; return r; }
    for (int64_t c = 0; c < n; ++c) list[c] = (uint64_t)c;

    double sumM = 0.0, sumS2 = 0.0, sumA = 0.0;
    for (int level = 0; level <= p->max_depth; ++level) {
        oracle_level* L = &r->level[level];
        L->n = n;
        L->uid = list;
        L->uid_hi = list_hi;
        L->m = (double*)malloc(sizeof(double) * (size_t)n);
        L->s = (double*)malloc(sizeof(double) * (size_t)n);
        L->I = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n1);
        L->sa = (double*)malloc(sizeof(double) * (size_t)n);
        L->sel = (uint8_t*)calloc((size_t)n, 1);
        if (!L->m || !L->s || !L->I || !L->sa || !L->sel) { r->status = OR_ENOMEM; return r; }
        r->levels_run = level + 1;

        /* direct MC with n1 trials in every sub-domain of the list */
        for (int64_t c = 0; c < n; ++c) {
            if (oracle_cube_w(p, level, list[c], list_hi[c], &L->I[c * n1], &L->m[c], &L->s[c], &L->sa[c]) != OR_OK)
                r->status = OR_ENONFINITE;
        }
        r->n_samples += (uint64_t)n * (uint64_t)n1 * (uint64_t)p->samples;
        r->n_cubes += (uint64_t)n;
        if (r->status != OR_OK) return r;

        /* threshold over this level's list (or over each parent's children)
         * and selection */
        L->min_margin = INFINITY;
        if (level < p->max_depth) {
            const int64_t group = (p->scope == 1 && level > 0) ? (int64_t)ipow_u64((uint64_t)p->split, D) : n;
            L->thr = oracle_threshold(L->s, n, p->sigma_mult, &L->mu, &L->sd);
            if (group != n) L->thr = L->mu = L->sd = NAN; /* no single threshold */
            double thr = 0.0;
            for (int64_t c = 0; c < n; ++c) {
                if (c % group == 0) thr = oracle_threshold(&L->s[c], group, p->sigma_mult, NULL, NULL);
                int sel = L->s[c] > thr;
                if (thr > 0.0) {
                    double margin = fabs(L->s[c] - thr) / thr;
                    if (margin < L->min_margin) L->min_margin = margin;
                    if (margin <= band_eps) {
                        int dec;
                        L->n_in_band++;
                        if (replay_lookup(rp, level, wide_id(list[c], list_hi[c]), &dec)) {
                            if (dec != sel) L->n_replayed++;
                            sel = dec;
                        }
                    }
                }
                L->sel[c] = (uint8_t)sel;
                L->n_sel += sel;
            }
        } else {
            L->thr = NAN;
            L->mu = NAN;
            L->sd = NAN;
        }

        /* accept the cubes that are not split, in list order */
        for (int64_t c = 0; c < n; ++c) {
            if (!L->sel[c]) {
                sumM += L->m[c];
                sumS2 += L->s[c] * L->s[c];
                sumA += L->sa[c];
            }
        }
        if (L->n_sel == 0) break;

        /* rtol stop: the selected cubes' current estimates complete the sum */
        int stop = 0;
        if (p->rtol > 0.0) {
            double runM = sumM, runS2 = sumS2;
            for (int64_t c = 0; c < n; ++c)
                if (L->sel[c]) {
                    runM += L->m[c];
                    runS2 += L->s[c] * L->s[c];
                }
            if (sqrt(runS2 / (double)(n1 - 1)) <= p->rtol * fabs(runM)) {
                stop = 1;
                r->flags |= OR_F_RTOL_MET;
            }
        }
        const uint64_t kids = ipow_u64((uint64_t)p->split, D);
        uint64_t n_next = (uint64_t)L->n_sel * kids;
        if (!stop && n_next > (uint64_t)p->max_cubes_per_level) {
            stop = 1;
            r->flags |= OR_F_TRUNCATED;
        }
        if (stop) {
            for (int64_t c = 0; c < n; ++c)
                if (L->sel[c]) {
                    sumM += L->m[c];
                    sumS2 += L->s[c] * L->s[c];
                    sumA += L->sa[c];
                }
            break;
        }

        /* split the selected cubes: children in parent order, c ascending */
        uint64_t* next = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n_next);
        uint32_t* next_hi = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n_next);
        if (!next || !next_hi) { free(next); free(next_hi); r->status = OR_ENOMEM; return r; }
        int64_t w = 0;
        for (int64_t c = 0; c < n; ++c)
            if (L->sel[c]) {
                oracle_children_w(list[c], list_hi[c], D, p->split, &next[w], &next_hi[w]);
                w += (int64_t)kids;
            }
        list = next;
        list_hi = next_hi;
        n = (int64_t)n_next;
    }
    r->integral = sumM;
    r->std = sqrt(sumS2);
    r->stderr_ = sqrt(sumS2 / (double)(n1 - 1));
    r->sum_abs = sumA;
    return r;
}

/* Flat accessors so that a caller without this file's struct layout (e.g. a
 * ctypes binding) can read a run. */
int oracle_run_status(const oracle_run* r) { return r->status; }
int oracle_run_flags(const oracle_run* r) { return r->flags; }
int oracle_run_levels(const oracle_run* r) { return r->levels_run; }
void oracle_run_totals(const oracle_run* r, double* out4, uint64_t* counts2)
{
    out4[0] = r->integral;
    out4[1] = r->std;
    out4[2] = r->stderr_;
    out4[3] = r->sum_abs;
    counts2[0] = r->n_samples;
    counts2[1] = r->n_cubes;
}
int64_t oracle_level_n(const oracle_run* r, int l) { return r->level[l].n; }
const uint64_t* oracle_level_uid(const oracle_run* r, int l) { return r->level[l].uid; }
const uint32_t* oracle_level_uid_hi(const oracle_run* r, int l) { return r->level[l].uid_hi; }
const double* oracle_level_m(const oracle_run* r, int l) { return r->level[l].m; }
const double* oracle_level_s(const oracle_run* r, int l) { return r->level[l].s; }
const double* oracle_level_I(const oracle_run* r, int l) { return r->level[l].I; }
const double* oracle_level_sa(const oracle_run* r, int l) { return r->level[l].sa; }
const uint8_t* oracle_level_sel(const oracle_run* r, int l) { return r->level[l].sel; }
void oracle_level_stats(const oracle_run* r, int l, double* out4, int64_t* counts3)
{
    out4[0] = r->level[l].thr;
    out4[1] = r->level[l].mu;
    out4[2] = r->level[l].sd;
    out4[3] = r->level[l].min_margin;
    counts3[0] = r->level[l].n_sel;
    counts3[1] = r->level[l].n_in_band;
    counts3[2] = r->level[l].n_replayed;
}
int oracle_sizeof_problem(void) { return (int)sizeof(oracle_problem); }
