// Exact hafnians and loop hafnians of integer matrices: the subset sum of
// Sec. 3.2 (Eq. Pset) over several prime fields on the GPU, then Chinese
// remaindering on the host.  Every term f(Z) counts tangles (an integer,
// Sec. 3.2) and the power-trace route of App. B needs only field operations,
// so the residues are exact and the reconstruction is exact once the product
// of the primes exceeds twice a bound on |haf|.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "haf_modp.hpp"
#include "haf_runtime.hpp"

namespace hafgpu {

constexpr int kModpMaxPrimes = 10;
constexpr int64_t kModpChunk = 1 << 18;     // subsets per coefficient launch
constexpr int kExactLimbs = 8;              // 256-bit magnitude

static bool is_prime(uint32_t p) {
    if (p < 2) return false;
    if (p % 2 == 0) return p == 2;
    for (uint32_t d = 3; d * d <= p; d += 2)
        if (p % d == 0) return false;
    return true;
}

static uint64_t pow_mod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = r * a % p;
        a = a * a % p;
        e >>= 1;
    }
    return r;
}

// The largest primes below 2^25, from the top.
static const std::vector<uint32_t>& default_primes() {
    static std::vector<uint32_t> ps;
    static std::once_flag once;
    std::call_once(once, [] {
        for (uint32_t p = kModpPrimeLimit - 1; ps.size() < (size_t)kModpMaxPrimes + 1; p -= 2)
            if (is_prime(p)) ps.push_back(p);
    });
    return ps;
}

static ModpPrime make_prime(uint32_t p) {
    ModpPrime P{};
    P.p = (double)p;
    P.pinv = 1.0 / (double)p;
    P.inv[0] = 0.0;
    for (int k = 1; k < 2 * kModpMaxN + 2; ++k) P.inv[k] = (double)pow_mod((uint64_t)k, p - 2, p);
    return P;
}

struct ModpWS {
    double* Ap = nullptr; size_t Ap_cap = 0;
    ModpPrime* pr = nullptr; size_t pr_cap = 0;
    double* coef = nullptr; size_t coef_cap = 0;
    double* part = nullptr; size_t part_cap = 0;
    double* res = nullptr; size_t res_cap = 0;
    hipStream_t st = nullptr;
};
static std::mutex g_modp_mu;
static ModpWS g_modp_ws[64];

// Residues of haf / lhaf of the even-size integer matrix A (dense, n x n) modulo
// each prime (validated by the caller: odd primes n + 1 < p < 2^25).
static int modp_residues(const int64_t* A, int n, int kind, const uint32_t* primes, int nprimes, uint32_t* out) {
    int dev = 0;
    int rc = ensure_device(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_modp_mu);
    ModpWS& w = g_modp_ws[dev];
    if (!w.st && hipStreamCreateWithFlags(&w.st, hipStreamNonBlocking) != hipSuccess)
        return set_error(HAF_E_DEVICE, "hipStreamCreate failed");
    hipStream_t st = w.st;
    const int N = n / 2;
    const bool loops = kind == HAF_KIND_LHAF;
    if (N == 0) {
        for (int i = 0; i < nprimes; ++i) out[i] = 1u;
        return HAF_OK;
    }
    const Plan plan = make_plan(n, kind, kModpChunk);
    const int64_t cstride = plan.max_chunk;
    const int64_t prime_stride = cstride * plan.ncoef;
    std::vector<double> hA((size_t)nprimes * n * n);
    std::vector<ModpPrime> hP((size_t)nprimes);
    for (int i = 0; i < nprimes; ++i) {
        hP[(size_t)i] = make_prime(primes[i]);
        const int64_t p = primes[i];
        for (int e = 0; e < n * n; ++e) {
            int64_t v = A[e] % p;
            hA[(size_t)i * n * n + e] = (double)(v < 0 ? v + p : v);
        }
    }
    if ((rc = grow((void**)&w.Ap, &w.Ap_cap, sizeof(double) * hA.size(), st))) return rc;
    if ((rc = grow((void**)&w.pr, &w.pr_cap, sizeof(ModpPrime) * hP.size(), st))) return rc;
    if ((rc = grow((void**)&w.coef, &w.coef_cap, sizeof(double) * (size_t)prime_stride * nprimes, st))) return rc;
    if ((rc = grow((void**)&w.part, &w.part_cap, sizeof(double) * (size_t)plan.nslots * nprimes, st))) return rc;
    if ((rc = grow((void**)&w.res, &w.res_cap, sizeof(double) * (size_t)nprimes, st))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(w.Ap, hA.data(), sizeof(double) * hA.size(), hipMemcpyHostToDevice, st),
                        "matrix upload")))
        return rc;
    if ((rc = hip_check(hipMemcpyAsync(w.pr, hP.data(), sizeof(ModpPrime) * hP.size(), hipMemcpyHostToDevice, st),
                        "prime upload")))
        return rc;
    const int grid = device_cus(dev) * 16;
    for (const Chunk& c : plan.chunks) {
        const int pidx = prof_begin(st, 0, 0.0, (int64_t)c.count * nprimes);
        rc = hip_check(launch_modp_coef(2 * c.m, loops, grid, nprimes, st, w.Ap, n, N, c.m, c.rank0, c.count, w.pr,
                                        w.coef, c.count, prime_stride),
                       "modular coefficient kernel launch");
        prof_end(pidx, st);
        if (rc) return rc;
        if ((rc = hip_check(launch_modp_series(loops, c.count, N, ((N - c.m) & 1) != 0, nprimes, st, w.coef, c.count,
                                               prime_stride, w.pr, w.part, c.slot0, plan.nslots),
                            "modular series kernel launch")))
            return rc;
    }
    if ((rc = hip_check(launch_modp_reduce(nprimes, st, w.part, plan.nslots, plan.nslots, w.pr, w.res),
                        "modular reduce kernel launch")))
        return rc;
    std::vector<double> hr((size_t)nprimes);
    if ((rc = hip_check(hipMemcpyAsync(hr.data(), w.res, sizeof(double) * nprimes, hipMemcpyDeviceToHost, st),
                        "residue download")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "stream synchronize"))) return rc;
    for (int i = 0; i < nprimes; ++i) out[i] = (uint32_t)hr[(size_t)i];
    return HAF_OK;
}

// Dense even-size copy (odd-n loop hafnian: A (+) [1]); checks symmetry (haf:
// off the diagonal only, the diagonal is ignored) and returns the largest
// |off-diagonal| and |diagonal| entries.
static int dense_copy(const int64_t* A, int n, int lda, int kind, std::vector<int64_t>* out, int* n_out,
                      double* moff, double* mdiag) {
    *moff = 0.0;
    *mdiag = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int64_t a = A[(int64_t)i * lda + j];
            if (a == INT64_MIN) return set_error(HAF_E_INVALID_ARG, "entry (%d, %d) is INT64_MIN", i, j);
            if (i != j && a != A[(int64_t)j * lda + i])
                return set_error(HAF_E_NOT_SYMMETRIC, "A[%d][%d] != A[%d][%d]", i, j, j, i);
            if (i != j) *moff = std::max(*moff, std::fabs((double)a));
            else if (kind == HAF_KIND_LHAF) *mdiag = std::max(*mdiag, std::fabs((double)a));
        }
    const int ne = (n % 2 == 1) ? n + 1 : n;
    out->assign((size_t)ne * ne, 0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) (*out)[(size_t)i * ne + j] = (i == j && kind == HAF_KIND_HAF) ? 0 : A[(int64_t)i * lda + j];
    if (ne != n) {
        (*out)[(size_t)n * ne + n] = 1;
        *mdiag = std::max(*mdiag, 1.0);
    }
    *n_out = ne;
    return HAF_OK;
}

// log2 of a bound on |haf| (matchings (n-1)!! times M_off^(n/2)) or |lhaf|
// (single-pair matchings T(n) times max(sqrt(M_off), M_diag)^n).
static double log2_bound(int n, int kind, double moff, double mdiag) {
    if (kind == HAF_KIND_HAF) {
        double l = 0.0;
        for (int k = n - 1; k > 1; k -= 2) l += std::log2((double)k);
        return l + (moff > 0.0 ? 0.5 * n * std::log2(moff) : -1e9);
    }
    long double t0 = 1.0L, t1 = 1.0L;                   // T(0), T(1); T(k) = T(k-1) + (k-1) T(k-2)
    for (int k = 2; k <= n; ++k) {
        const long double t2 = t1 + (long double)(k - 1) * t0;
        t0 = t1;
        t1 = t2;
    }
    const double m = std::max({ std::sqrt(moff), mdiag, 1.0 });
    return (double)std::log2(n >= 1 ? t1 : 1.0L) + n * std::log2(m);
}

// ---------------------------------------------------------------- little big-integer helpers (32-bit limbs)
static void big_mul_add(uint32_t* v, int limbs, uint32_t mul, uint32_t add) {
    uint64_t carry = add;
    for (int i = 0; i < limbs; ++i) {
        const uint64_t t = (uint64_t)v[i] * mul + carry;
        v[i] = (uint32_t)t;
        carry = t >> 32;
    }
}
static int big_cmp(const uint32_t* a, const uint32_t* b, int limbs) {
    for (int i = limbs - 1; i >= 0; --i)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}
static void big_sub(uint32_t* a, const uint32_t* b, int limbs) {   // a -= b, a >= b
    int64_t borrow = 0;
    for (int i = 0; i < limbs; ++i) {
        int64_t t = (int64_t)a[i] - b[i] - borrow;
        borrow = t < 0;
        a[i] = (uint32_t)(t + (borrow ? ((int64_t)1 << 32) : 0));
    }
}
static uint32_t big_mod(const uint32_t* v, int limbs, uint32_t p) {
    uint64_t r = 0;
    for (int i = limbs - 1; i >= 0; --i) r = ((r << 32) | v[i]) % p;
    return (uint32_t)r;
}

// Garner's mixed-radix reconstruction: v in [0, M), M = prod p_i, as limbs;
// then the symmetric representative (|v| <= M/2) as sign and magnitude.
static void crt_symmetric(const uint32_t* r, const uint32_t* p, int k, uint32_t* mag, int* sign) {
    std::vector<uint64_t> d((size_t)k);
    for (int i = 0; i < k; ++i) {
        uint64_t t = r[i] % p[i];
        for (int j = 0; j < i; ++j) {
            t = (t + p[i] - d[(size_t)j] % p[i]) % p[i];
            t = t * pow_mod(p[j] % p[i], p[i] - 2, p[i]) % p[i];
        }
        d[(size_t)i] = t;
    }
    // Horner from the top digit: v = d_(k-1); v = v p_i + d_i
    uint32_t v[kExactLimbs + 1] = {}, M[kExactLimbs + 1] = {};
    v[0] = (uint32_t)d[(size_t)k - 1];
    for (int i = k - 2; i >= 0; --i) big_mul_add(v, kExactLimbs + 1, p[i], (uint32_t)d[(size_t)i]);
    M[0] = 1;
    for (int i = 0; i < k; ++i) big_mul_add(M, kExactLimbs + 1, p[i], 0);
    uint32_t twice[kExactLimbs + 1];
    std::memcpy(twice, v, sizeof v);
    big_mul_add(twice, kExactLimbs + 1, 2, 0);
    *sign = 1;
    if (big_cmp(twice, M, kExactLimbs + 1) > 0) {   // v > M/2: negative value v - M
        uint32_t t[kExactLimbs + 1];
        std::memcpy(t, M, sizeof M);
        big_sub(t, v, kExactLimbs + 1);
        std::memcpy(v, t, sizeof t);
        *sign = -1;
    }
    for (int i = 0; i < kExactLimbs; ++i) mag[i] = v[i];
}

}  // namespace hafgpu

using namespace hafgpu;

extern "C" {

int haf_modp_c(const int64_t* A, int n, int lda, int kind, const uint32_t* primes, int nprimes, uint32_t* residues) {
    clear_error();
    if (!A || !primes || !residues) return set_error(HAF_E_INVALID_ARG, "null pointer");
    if (n < 0 || (n > 0 && lda < n)) return set_error(HAF_E_INVALID_ARG, "bad n = %d / lda = %d", n, lda);
    if (kind != HAF_KIND_HAF && kind != HAF_KIND_LHAF) return set_error(HAF_E_INVALID_ARG, "unknown kind %d", kind);
    if (nprimes < 1 || nprimes > kModpMaxPrimes)
        return set_error(HAF_E_INVALID_ARG, "nprimes = %d not in 1..%d", nprimes, kModpMaxPrimes);
    const int ne = (n % 2 == 1 && kind == HAF_KIND_LHAF) ? n + 1 : n;
    if (ne > HAF_MAX_N) return set_error(HAF_E_TOO_LARGE, "n = %d exceeds the limit %d", n, HAF_MAX_N);
    for (int i = 0; i < nprimes; ++i)
        if (primes[i] <= (uint32_t)ne + 1 || primes[i] >= kModpPrimeLimit || !is_prime(primes[i]))
            return set_error(HAF_E_INVALID_ARG, "primes[%d] = %u is not a prime in (n + 1, 2^25)", i, primes[i]);
    std::vector<int64_t> Ad;
    int nd = 0;
    double moff, mdiag;
    int rc = dense_copy(A, n, lda, kind, &Ad, &nd, &moff, &mdiag);
    if (rc) return rc;
    if (n % 2 == 1 && kind == HAF_KIND_HAF) {
        for (int i = 0; i < nprimes; ++i) residues[i] = 0u;
        return HAF_OK;
    }
    return modp_residues(Ad.data(), nd, kind, primes, nprimes, residues);
}

int haf_exact_i64(const int64_t* A, int n, int lda, int kind, uint32_t* magnitude, int* sign) {
    clear_error();
    if (!A || !magnitude || !sign) return set_error(HAF_E_INVALID_ARG, "null pointer");
    if (n < 0 || (n > 0 && lda < n)) return set_error(HAF_E_INVALID_ARG, "bad n = %d / lda = %d", n, lda);
    if (kind != HAF_KIND_HAF && kind != HAF_KIND_LHAF) return set_error(HAF_E_INVALID_ARG, "unknown kind %d", kind);
    const int ne = (n % 2 == 1 && kind == HAF_KIND_LHAF) ? n + 1 : n;
    if (ne > HAF_MAX_N) return set_error(HAF_E_TOO_LARGE, "n = %d exceeds the limit %d", n, HAF_MAX_N);
    std::memset(magnitude, 0, sizeof(uint32_t) * kExactLimbs);
    *sign = 1;
    std::vector<int64_t> Ad;
    int nd = 0;
    double moff, mdiag;
    int rc = dense_copy(A, n, lda, kind, &Ad, &nd, &moff, &mdiag);
    if (rc) return rc;
    if (n % 2 == 1 && kind == HAF_KIND_HAF) {
        *sign = 0;
        return HAF_OK;
    }
    if (nd == 0) {
        magnitude[0] = 1;
        return HAF_OK;
    }
    // enough primes for |value| <= 2^lb, so that M > 2 |value| + 1, plus one check prime
    const double lb = log2_bound(nd, kind, moff, mdiag);
    const std::vector<uint32_t>& ps = default_primes();
    double bits = 0.0;
    int k = 0;
    while (k < kModpMaxPrimes && (k == 0 || bits < lb + 2.0)) bits += std::log2((double)ps[(size_t)k++]);
    if (bits < lb + 2.0 || lb + 2.0 > 32.0 * kExactLimbs - 2.0)
        return set_error(HAF_E_TOO_LARGE, "the bound 2^%.1f on the result needs more than %d primes", lb,
                         kModpMaxPrimes);
    std::vector<uint32_t> res((size_t)k + 1);
    if ((rc = modp_residues(Ad.data(), nd, kind, ps.data(), k + 1, res.data()))) return rc;
    crt_symmetric(res.data(), ps.data(), k, magnitude, sign);
    // the check prime must agree with the reconstruction
    const uint32_t pc = ps[(size_t)k];
    uint32_t m = big_mod(magnitude, kExactLimbs, pc);
    if (*sign < 0 && m != 0) m = pc - m;
    if (m != res[(size_t)k])
        return set_error(HAF_E_DEVICE, "check prime %u disagrees with the reconstruction (%u vs %u)", pc, m,
                         res[(size_t)k]);
    bool zero = true;
    for (int i = 0; i < kExactLimbs; ++i) zero = zero && magnitude[i] == 0;
    if (zero) *sign = 0;
    return HAF_OK;
}

}  // extern "C"
