/*
 * CPU oracle for the hafnian and loop hafnian -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code with the GPU library.
 *
 * Routes (all plain and slow on purpose):
 *   brute force   haf / lhaf straight from the definitions (Sec. 2, Eq. hafA and
 *                 the loop-hafnian sum over single-pair matchings), by expanding
 *                 along the lowest remaining vertex with a table over vertex sets;
 *   formula       the inclusion-exclusion sum of Sec. 3.2-3.3 with power traces
 *                 taken from explicit matrix powers (no Schur form, no
 *                 characteristic polynomial), in double, long double,
 *                 double-double or binary128;
 *   mod p         the same sum over the prime field F_p for integer matrices
 *                 (each f(Z) counts tangles, so it is an integer), with the traces
 *                 from a Hessenberg form by Gaussian elimination and the
 *                 characteristic-polynomial recurrence of App. B's setting;
 *   ryser         permanents, for the bipartite identity of Sec. 1.1.
 *
 * Matrices are row-major interleaved complex double (re, im) with leading
 * dimension n unless stated otherwise.  Results are returned as (hi, lo) double
 * pairs per component so extended precision survives the trip to Python.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <quadmath.h>

/* ------------------------------------------------------------------ */
/* double-double arithmetic (Dekker / Knuth error-free transformations) */
typedef struct { double hi, lo; } dd_t;
static inline dd_t dd_two_sum(double a, double b) {
    double s = a + b, bb = s - a;
    dd_t r = { s, (a - (s - bb)) + (b - bb) };
    return r;
}
static inline dd_t dd_quick(double a, double b) { double s = a + b; dd_t r = { s, b - (s - a) }; return r; }
static inline dd_t dd_add(dd_t a, dd_t b) {
    dd_t s = dd_two_sum(a.hi, b.hi), t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi; s = dd_quick(s.hi, s.lo); s.lo += t.lo; return dd_quick(s.hi, s.lo);
}
static inline dd_t dd_neg(dd_t a) { dd_t r = { -a.hi, -a.lo }; return r; }
static inline dd_t dd_sub(dd_t a, dd_t b) { return dd_add(a, dd_neg(b)); }
static inline dd_t dd_mul(dd_t a, dd_t b) {
    double p = a.hi * b.hi, e = fma(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    return dd_quick(p, e);
}
static inline dd_t dd_divd(dd_t a, double b) {   /* a / b by one Newton correction */
    double q1 = a.hi / b;
    double p = q1 * b, e = fma(q1, b, -p);
    dd_t r = dd_sub(a, dd_quick(p, e));
    double q2 = r.hi / b;
    return dd_quick(q1, q2);
}
static inline dd_t dd_fromd(double x) { dd_t r = { x, 0.0 }; return r; }

/* ---------------- instantiate the generic body per precision ---------------- */
#define F_ACC_SIGNED(sr, si, f, neg)                                                       \
    do {                                                                                   \
        if (neg) { F(acc_add)(&(sr), T_NEG((f).re)); F(acc_add)(&(si), T_NEG((f).im)); } \
        else { F(acc_add)(&(sr), (f).re); F(acc_add)(&(si), (f).im); }                     \
    } while (0)

/* double */
#define T double
#define F(x) x##_d
#define T_ADD(a, b) ((a) + (b))
#define T_SUB(a, b) ((a) - (b))
#define T_MUL(a, b) ((a) * (b))
#define T_DIVI(a, k) ((a) / (double)(k))
#define T_NEG(a) (-(a))
#define T_FROMD(x) (x)
#define T_HI(x) ((double)(x))
#define T_LO(x) (0.0)
#define T_ZERO 0.0
#define T_ONE 1.0
#include "formula_body.inc"
#undef T
#undef F
#undef T_ADD
#undef T_SUB
#undef T_MUL
#undef T_DIVI
#undef T_NEG
#undef T_FROMD
#undef T_HI
#undef T_LO
#undef T_ZERO
#undef T_ONE

/* long double (x87 80-bit) */
#define T long double
#define F(x) x##_ld
#define T_ADD(a, b) ((a) + (b))
#define T_SUB(a, b) ((a) - (b))
#define T_MUL(a, b) ((a) * (b))
#define T_DIVI(a, k) ((a) / (long double)(k))
#define T_NEG(a) (-(a))
#define T_FROMD(x) ((long double)(x))
#define T_HI(x) ((double)(x))
#define T_LO(x) ((double)((x) - (long double)(double)(x)))
#define T_ZERO 0.0L
#define T_ONE 1.0L
#include "formula_body.inc"
#undef T
#undef F
#undef T_ADD
#undef T_SUB
#undef T_MUL
#undef T_DIVI
#undef T_NEG
#undef T_FROMD
#undef T_HI
#undef T_LO
#undef T_ZERO
#undef T_ONE

/* double-double */
#define T dd_t
#define F(x) x##_dd
#define T_ADD(a, b) dd_add((a), (b))
#define T_SUB(a, b) dd_sub((a), (b))
#define T_MUL(a, b) dd_mul((a), (b))
#define T_DIVI(a, k) dd_divd((a), (double)(k))
#define T_NEG(a) dd_neg(a)
#define T_FROMD(x) dd_fromd(x)
#define T_HI(x) ((x).hi)
#define T_LO(x) ((x).lo)
#define T_ZERO ((dd_t){ 0.0, 0.0 })
#define T_ONE ((dd_t){ 1.0, 0.0 })
#include "formula_body.inc"
#undef T
#undef F
#undef T_ADD
#undef T_SUB
#undef T_MUL
#undef T_DIVI
#undef T_NEG
#undef T_FROMD
#undef T_HI
#undef T_LO
#undef T_ZERO
#undef T_ONE

/* IEEE binary128 (software) */
#define T __float128
#define F(x) x##_q
#define T_ADD(a, b) ((a) + (b))
#define T_SUB(a, b) ((a) - (b))
#define T_MUL(a, b) ((a) * (b))
#define T_DIVI(a, k) ((a) / (__float128)(k))
#define T_NEG(a) (-(a))
#define T_FROMD(x) ((__float128)(x))
#define T_HI(x) ((double)(x))
#define T_LO(x) ((double)((x) - (__float128)(double)(x)))
#define T_ZERO ((__float128)0)
#define T_ONE ((__float128)1)
#include "formula_body.inc"
#undef T
#undef F
#undef T_ADD
#undef T_SUB
#undef T_MUL
#undef T_DIVI
#undef T_NEG
#undef T_FROMD
#undef T_HI
#undef T_LO
#undef T_ZERO
#undef T_ONE

/* precision codes shared with the Python side */
enum { ORC_D = 0, ORC_LD = 1, ORC_DD = 2, ORC_Q = 3 };

int orc_formula_range(const double* A, int n, int loops, int prec, uint64_t lo, uint64_t hi,
                      int nthreads, double* out, double* absum) {
    if (n < 0 || (n & 1) || n > 64 || lo > hi) return -1;
    switch (prec) {
    case ORC_D: return range_sum_d(A, n, loops, lo, hi, nthreads, out, absum);
    case ORC_LD: return range_sum_ld(A, n, loops, lo, hi, nthreads, out, absum);
    case ORC_DD: return range_sum_dd(A, n, loops, lo, hi, nthreads, out, absum);
    case ORC_Q: return range_sum_q(A, n, loops, lo, hi, nthreads, out, absum);
    }
    return -1;
}

int orc_formula_masks(const double* A, int n, int loops, int prec, const uint32_t* masks, int64_t count,
                      int nthreads, double* out) {
    if (n < 0 || (n & 1) || n > 64) return -1;
    switch (prec) {
    case ORC_D: return mask_sum_d(A, n, loops, masks, count, nthreads, out);
    case ORC_LD: return mask_sum_ld(A, n, loops, masks, count, nthreads, out);
    case ORC_DD: return mask_sum_dd(A, n, loops, masks, count, nthreads, out);
    case ORC_Q: return mask_sum_q(A, n, loops, masks, count, nthreads, out);
    }
    return -1;
}

int orc_term(const double* A, int n, int loops, int prec, uint32_t mask, double* out) {
    if (n < 0 || (n & 1) || n > 64) return -1;
    switch (prec) {
    case ORC_D: return one_term_d(A, n, loops, mask, out);
    case ORC_LD: return one_term_ld(A, n, loops, mask, out);
    case ORC_DD: return one_term_dd(A, n, loops, mask, out);
    case ORC_Q: return one_term_q(A, n, loops, mask, out);
    }
    return -1;
}

int orc_ryser(const double* W, int k, int prec, int nthreads, double* out) {
    if (k < 0 || k > 40) return -1;
    switch (prec) {
    case ORC_D: return ryser_d(W, k, nthreads, out);
    case ORC_LD: return ryser_ld(W, k, nthreads, out);
    case ORC_DD: return ryser_dd(W, k, nthreads, out);
    case ORC_Q: return ryser_q(W, k, nthreads, out);
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Brute force from the definitions.
 * val[S] = sum over matchings of the vertex set S.  The lowest vertex i of S
 * is either matched to some j in S (weight A_ij) or, for the loop hafnian,
 * covered by its loop (weight A_ii).  Every proper subset of S is numerically
 * smaller than S, so one increasing sweep over all masks fills the table.   */
int orc_brute(const double* A, int n, int loops, double* out) {
    if (n < 0 || n > 24) return -1;
    size_t M = (size_t)1 << n;
    long double* re = (long double*)malloc(sizeof(long double) * M);
    long double* im = (long double*)malloc(sizeof(long double) * M);
    if (!re || !im) { free(re); free(im); return -1; }
    re[0] = 1.0L; im[0] = 0.0L;
    for (size_t S = 1; S < M; S++) {
        int i = __builtin_ctzll((unsigned long long)S);
        size_t rest = S & ~((size_t)1 << i);
        long double sr = 0.0L, si = 0.0L;
        if (loops) {
            long double ar = A[2 * (i * n + i)], ai = A[2 * (i * n + i) + 1];
            sr += ar * re[rest] - ai * im[rest];
            si += ar * im[rest] + ai * re[rest];
        }
        for (size_t m = rest; m; m &= m - 1) {
            int j = __builtin_ctzll((unsigned long long)m);
            size_t sub = rest & ~((size_t)1 << j);
            long double ar = A[2 * (i * n + j)], ai = A[2 * (i * n + j) + 1];
            sr += ar * re[sub] - ai * im[sub];
            si += ar * im[sub] + ai * re[sub];
        }
        re[S] = sr; im[S] = si;
    }
    long double vr = re[M - 1], vi = im[M - 1];
    out[0] = (double)vr; out[1] = (double)(vr - (long double)(double)vr);
    out[2] = (double)vi; out[3] = (double)(vi - (long double)(double)vi);
    free(re); free(im);
    return 0;
}

/* Exact brute force for integer matrices (int64 entries, 128-bit sums).
 * Writes the signed 128-bit result as (low 64 bits, high 64 bits).          */
int orc_brute_int(const int64_t* A, int n, int loops, uint64_t* out) {
    if (n < 0 || n > 24) return -1;
    size_t M = (size_t)1 << n;
    __int128* v = (__int128*)malloc(sizeof(__int128) * M);
    if (!v) return -1;
    v[0] = 1;
    for (size_t S = 1; S < M; S++) {
        int i = __builtin_ctzll((unsigned long long)S);
        size_t rest = S & ~((size_t)1 << i);
        __int128 acc = 0;
        if (loops) acc += (__int128)A[i * n + i] * v[rest];
        for (size_t m = rest; m; m &= m - 1) {
            int j = __builtin_ctzll((unsigned long long)m);
            acc += (__int128)A[i * n + j] * v[rest & ~((size_t)1 << j)];
        }
        v[S] = acc;
    }
    unsigned __int128 u = (unsigned __int128)v[M - 1];
    out[0] = (uint64_t)u; out[1] = (uint64_t)(u >> 64);
    free(v);
    return 0;
}

/* ------------------------------------------------------------------ */
/* The formula over F_p (p an odd prime < 2^31, p > n).                  */
typedef struct { uint64_t p, m; } modp_t;   /* m = floor(2^64 / p) for Barrett reduction */
static inline uint64_t mp_red(const modp_t* F, uint64_t x) {   /* x < p^2 */
    uint64_t q = (uint64_t)(((unsigned __int128)x * F->m) >> 64);
    uint64_t r = x - q * F->p;
    return r >= F->p ? r - F->p : r;
}
static inline uint64_t mp_mul(const modp_t* F, uint64_t a, uint64_t b) { return mp_red(F, a * b); }
static inline uint64_t mp_add(const modp_t* F, uint64_t a, uint64_t b) { uint64_t s = a + b; return s >= F->p ? s - F->p : s; }
static inline uint64_t mp_sub(const modp_t* F, uint64_t a, uint64_t b) { return a >= b ? a - b : a + F->p - b; }
static uint64_t mp_pow(const modp_t* F, uint64_t a, uint64_t e) {
    uint64_t r = 1 % F->p;
    while (e) { if (e & 1) r = mp_mul(F, r, a); a = mp_mul(F, a, a); e >>= 1; }
    return r;
}
static inline uint64_t mp_inv(const modp_t* F, uint64_t a) { return mp_pow(F, a, F->p - 2); }

/*
 * f(Z) mod p.  B as in the complex formula (X*A with zero diagonal on the
 * subset).  Traces: reduce B to upper Hessenberg form by similarity with
 * elementary (Gauss) transformations, pivoting on any nonzero entry; take the
 * characteristic polynomial of the Hessenberg form by the recurrence over its
 * leading principal blocks; turn coefficients into power sums by Newton's
 * identities (App. B notes the traces follow from the polynomial).
 */
static uint64_t modp_term(const modp_t* F, const uint64_t* Am, int n, int loops, uint32_t mask,
                          uint64_t* H, uint64_t* cp, uint64_t* tr, uint64_t* ell, uint64_t* y, uint64_t* y2,
                          int* idx, const uint64_t* inv_small) {
    int N = n / 2, s = 0;
    for (int i = 0; i < N; i++)
        if (mask >> i & 1u) { idx[s++] = 2 * i; idx[s++] = 2 * i + 1; }
    if (s == 0 || N == 0) return 0;
    uint64_t p = F->p;
    for (int r = 0; r < s; r++)
        for (int c = 0; c < s; c++) {
            int row = idx[r] ^ 1, col = idx[c];
            H[r * s + c] = (row == col) ? 0 : Am[row * n + col];
        }
    if (loops) {   /* l_k = d^T B^(k-1) X d, before B is overwritten */
        for (int r = 0; r < s; r++) y[r] = Am[idx[r ^ 1] * n + idx[r ^ 1]];
        for (int k = 1; k <= N; k++) {
            uint64_t acc = 0;
            for (int r = 0; r < s; r++) acc = mp_add(F, acc, mp_mul(F, Am[idx[r] * n + idx[r]], y[r]));
            ell[k] = acc;
            if (k < N) {
                for (int r = 0; r < s; r++) {
                    uint64_t t = 0;
                    for (int c = 0; c < s; c++) t = mp_add(F, t, mp_mul(F, H[r * s + c], y[c]));
                    y2[r] = t;
                }
                memcpy(y, y2, sizeof(uint64_t) * s);
            }
        }
    }
    /* Hessenberg form by stabilised elimination: for column j, bring a nonzero
     * entry of rows j+1.. to row j+1 (row + column swap), then clear rows j+2..
     * with L^{-1} on the left and L on the right.                             */
    for (int j = 0; j + 2 < s; j++) {
        int piv = -1;
        for (int r = j + 1; r < s; r++) if (H[r * s + j]) { piv = r; break; }
        if (piv < 0) continue;
        if (piv != j + 1) {
            for (int c = 0; c < s; c++) { uint64_t t = H[piv * s + c]; H[piv * s + c] = H[(j + 1) * s + c]; H[(j + 1) * s + c] = t; }
            for (int r = 0; r < s; r++) { uint64_t t = H[r * s + piv]; H[r * s + piv] = H[r * s + j + 1]; H[r * s + j + 1] = t; }
        }
        uint64_t ip = mp_inv(F, H[(j + 1) * s + j]);
        for (int r = j + 2; r < s; r++) {
            uint64_t l = mp_mul(F, H[r * s + j], ip);
            if (!l) continue;
            for (int c = j; c < s; c++) H[r * s + c] = mp_sub(F, H[r * s + c], mp_mul(F, l, H[(j + 1) * s + c]));
            for (int q = 0; q < s; q++) H[q * s + j + 1] = mp_add(F, H[q * s + j + 1], mp_mul(F, l, H[q * s + r]));
        }
    }
    /* c_i(x) = det(x I - H[0:i,0:i]);  c_i = (x - h_{i-1,i-1}) c_{i-1}
     *   - sum_{r<i-1} h_{r,i-1} (prod_{k=r+1}^{i-1} h_{k,k-1}) c_r.
     * cp holds c_i with coefficient of x^e at cp[i*(s+1) + e].               */
    memset(cp, 0, sizeof(uint64_t) * (size_t)(s + 1) * (s + 1));
    cp[0] = 1;
    for (int i = 1; i <= s; i++) {
        uint64_t* ci = cp + (size_t)i * (s + 1);
        const uint64_t* cm = cp + (size_t)(i - 1) * (s + 1);
        for (int e = 1; e <= i; e++) ci[e] = cm[e - 1];
        uint64_t hd = H[(i - 1) * s + i - 1];
        for (int e = 0; e < i; e++) ci[e] = mp_sub(F, ci[e], mp_mul(F, hd, cm[e]));
        uint64_t prod = 1;
        for (int r = i - 2; r >= 0; r--) {
            prod = mp_mul(F, prod, H[(r + 1) * s + r]);
            if (!prod) break;
            uint64_t g = mp_mul(F, H[r * s + i - 1], prod);
            const uint64_t* cr = cp + (size_t)r * (s + 1);
            for (int e = 0; e <= r; e++) ci[e] = mp_sub(F, ci[e], mp_mul(F, g, cr[e]));
        }
    }
    /* a_k = coefficient of x^(s-k);  Newton: p_k = -k a_k - sum_{i<k} a_i p_{k-i} */
    const uint64_t* cs = cp + (size_t)s * (s + 1);
    for (int k = 1; k <= N; k++) {
        uint64_t ak = k <= s ? cs[s - k] : 0;
        uint64_t acc = mp_sub(F, 0, mp_mul(F, (uint64_t)k % p, ak));
        for (int i = 1; i < k && i <= s; i++) acc = mp_sub(F, acc, mp_mul(F, cs[s - i], tr[k - i]));
        tr[k] = acc;
    }
    /* c_k = p_k/(2k) [+ l_k/2];  e_j = (1/j) sum_{k=1}^{j} k c_k e_{j-k};  f = e_N */
    uint64_t* e = y2;   /* reuse: needs N+1 <= n+1 entries */
    uint64_t* c = y;
    for (int k = 1; k <= N; k++) {
        uint64_t ck = mp_mul(F, tr[k], inv_small[2 * k]);
        if (loops) ck = mp_add(F, ck, mp_mul(F, ell[k], inv_small[2]));
        c[k] = ck;
    }
    e[0] = 1;
    for (int j = 1; j <= N; j++) {
        uint64_t acc = 0;
        for (int k = 1; k <= j; k++) acc = mp_add(F, acc, mp_mul(F, mp_mul(F, (uint64_t)k, c[k]), e[j - k]));
        e[j] = mp_mul(F, acc, inv_small[j]);
    }
    return e[N];
}

/* Signed sum over all subsets mod p.  A holds integer entries (int64).      */
int orc_modp(const int64_t* A, int n, int loops, uint64_t p, int nthreads, uint64_t* out) {
    if (n < 0 || (n & 1) || n > 62 || p < 3 || p >= (1ull << 31) || p <= (uint64_t)n + 1) return -1;
    int N = n / 2;
    modp_t F = { p, (uint64_t)(((unsigned __int128)1 << 64) / p) };
    uint64_t* Am = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n * n + 1));
    uint64_t inv_small[130];
    if (!Am) return -1;
    for (int i = 0; i < n * n; i++) {
        int64_t v = A[i] % (int64_t)p;
        Am[i] = (uint64_t)(v < 0 ? v + (int64_t)p : v);
    }
    inv_small[0] = 0;
    for (int k = 1; k < 130; k++) inv_small[k] = mp_inv(&F, (uint64_t)k % p);
    if (nthreads < 1) nthreads = 1;
    uint64_t total = ((uint64_t)1 << N);
    uint64_t* part = (uint64_t*)calloc((size_t)nthreads, sizeof(uint64_t));
    int ok = 1;
#pragma omp parallel num_threads(nthreads) reduction(&& : ok)
    {
        int t = omp_get_thread_num(), nt = omp_get_num_threads();
        uint64_t a = 1 + (total - 1) * t / nt, b = 1 + (total - 1) * (t + 1) / nt;
        uint64_t* H = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n * n + 1));
        uint64_t* cp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 1) * (n + 1));
        uint64_t* tr = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(N + 2));
        uint64_t* ell = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(N + 2));
        uint64_t* y = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 2));
        uint64_t* y2 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 2));
        int* idx = (int*)malloc(sizeof(int) * (size_t)(n + 1));
        uint64_t acc = 0;
        if (!H || !cp || !tr || !ell || !y || !y2 || !idx) ok = 0;
        else
            for (uint64_t m = a; m < b; m++) {
                uint64_t f = modp_term(&F, Am, n, loops, (uint32_t)m, H, cp, tr, ell, y, y2, idx, inv_small);
                acc = ((N - __builtin_popcountll(m)) & 1) ? mp_sub(&F, acc, f) : mp_add(&F, acc, f);
            }
        part[t] = acc;
        free(H); free(cp); free(tr); free(ell); free(y); free(y2); free(idx);
    }
    uint64_t acc = 0;
    for (int t = 0; t < nthreads; t++) acc = mp_add(&F, acc, part[t]);
    *out = (N == 0) ? 1 % p : acc;
    free(part); free(Am);
    return ok ? 0 : -1;
}

/* One term f(Z) mod p (for tests that pin single terms). */
int orc_modp_term(const int64_t* A, int n, int loops, uint64_t p, uint32_t mask, uint64_t* out) {
    if (n < 0 || (n & 1) || n > 62 || p < 3 || p >= (1ull << 31) || p <= (uint64_t)n + 1) return -1;
    int N = n / 2;
    modp_t F = { p, (uint64_t)(((unsigned __int128)1 << 64) / p) };
    uint64_t inv_small[130];
    inv_small[0] = 0;
    for (int k = 1; k < 130; k++) inv_small[k] = mp_inv(&F, (uint64_t)k % p);
    uint64_t* Am = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n * n + 1));
    uint64_t* H = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n * n + 1));
    uint64_t* cp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 1) * (n + 1));
    uint64_t* tr = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(N + 2));
    uint64_t* ell = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(N + 2));
    uint64_t* y = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 2));
    uint64_t* y2 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 2));
    int* idx = (int*)malloc(sizeof(int) * (size_t)(n + 1));
    int rc = -1;
    if (Am && H && cp && tr && ell && y && y2 && idx) {
        for (int i = 0; i < n * n; i++) {
            int64_t v = A[i] % (int64_t)p;
            Am[i] = (uint64_t)(v < 0 ? v + (int64_t)p : v);
        }
        *out = modp_term(&F, Am, n, loops, mask, H, cp, tr, ell, y, y2, idx, inv_small);
        rc = 0;
    }
    free(Am); free(H); free(cp); free(tr); free(ell); free(y); free(y2); free(idx);
    return rc;
}
