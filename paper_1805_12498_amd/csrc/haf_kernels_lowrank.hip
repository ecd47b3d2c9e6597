// Hafnians of low-rank matrices (App. C): for an n x r factor G, the hafnian of
// any matrix whose entries above the diagonal are those of G G^T is
//     haf = sum over even exponent vectors e (e_1 + .. + e_r = n, every e_j even)
//           of lambda_e prod_j (e_j - 1)!!,
// where lambda_p are the coefficients of q(x) = prod_(i=1..n) (sum_j g_ij x_j).
// The cost is polynomial in n times the number of monomials of degree n in r
// variables, C(n + r - 1, r - 1), instead of 2^(n/2).
//
// The expansion runs on the GPU one linear factor at a time: the coefficients
// of degree k are new[p] = sum_(j: p_j >= 1) g_kj old[p - e_j], one thread per
// monomial.  Monomials of degree k are numbered by the combinatorial number
// system over their bar positions b_i = p_1 + .. + p_i + i - 1 (i < r), an
// (r-1)-subset of {0 .. k+r-2}: rank(p) = sum_i C(b_i, i).  Removing one x_j
// lowers every bar to the right of x_j by one, so every neighbour's rank is a
// prefix sum of C(b_i, i) plus a suffix sum of C(b_i - 1, i).  The last step sums the even
// monomials with their double-factorial weights in double-double, by a fixed
// tree per block and the fixed-order fold of the partial slots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "haf_common.hpp"
#include "haf_launch.hpp"
#include "haf_runtime.hpp"

namespace hafgpu {

constexpr int kLowRankMaxR = 8;
constexpr int kBinA = 64 + kLowRankMaxR;       // binomials C(a, b) for a < kBinA, b <= kLowRankMaxR
constexpr int kBinB = kLowRankMaxR + 1;
constexpr int kLowRankBlock = 256;

__device__ __forceinline__ uint64_t binom_t(const uint64_t* __restrict__ tab, int a, int b) {
    return (a < b || a < 0) ? 0ull : tab[a * kBinB + b];
}

// bar positions of the monomial of rank `rank` (degree k, R variables)
template <int R>
__device__ __forceinline__ void unrank_bars(uint64_t rank, int k, const uint64_t* __restrict__ tab, int (&b)[R]) {
    int top = k + R - 2;                        // largest possible bar position
#pragma unroll
    for (int i = R - 1; i >= 1; --i) {
        int x = top;
        while (binom_t(tab, x, i) > rank) --x;
        b[i] = x;
        rank -= binom_t(tab, x, i);
        top = x - 1;
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_lowrank_step(const double2* __restrict__ G, int ldg, int k,
                                                      const uint64_t* __restrict__ tab,
                                                      const double2* __restrict__ old_c, double2* __restrict__ new_c,
                                                      int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const double2* g = G + (int64_t)(k - 1) * ldg;      // the k-th linear factor
    if (R == 1) {
        new_c[t] = cmul(g[0], old_c[0]);
        return;
    }
    int b[R];
    unrank_bars<R>((uint64_t)t, k, tab, b);
    // exponents from the bars (b_0 = -1, b_R = k + R - 1)
    int p[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int lo = j == 0 ? -1 : b[j];
        const int hi = j == R - 1 ? k + R - 1 : b[j + 1];
        p[j] = hi - lo - 1;
    }
    // rank of p - e_j (j 0-based, bars 1..R-1): sum_(i <= j) C(b_i, i) + sum_(i > j) C(b_i - 1, i)
    uint64_t pre[R], suf[R + 1];
    pre[0] = 0;
#pragma unroll
    for (int i = 1; i < R; ++i) pre[i] = pre[i - 1] + binom_t(tab, b[i], i);
    suf[R] = 0;
#pragma unroll
    for (int i = R - 1; i >= 1; --i) suf[i] = suf[i + 1] + binom_t(tab, b[i] - 1, i);
    double2 acc = cz();
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (p[j] < 1) continue;
        // variable j (0-based) sits between bars j and j+1; removing it lowers bars j+1..R-1
        const uint64_t rk = pre[j] + (j + 1 <= R - 1 ? suf[j + 1] : 0ull);
        cfma(acc, g[j], old_c[rk]);
    }
    new_c[t] = acc;
}

// Even monomials of degree n times prod_j (p_j - 1)!!, summed in double-double per
// block (fixed tree); also the block's sum of |terms| (double) for the condition number.
template <int R>
__global__ __launch_bounds__(kLowRankBlock) void k_lowrank_even_sum(const double2* __restrict__ c, int n,
                                                                    const uint64_t* __restrict__ tab, int64_t count,
                                                                    double* __restrict__ partials,
                                                                    double* __restrict__ abs_partials) {
    __shared__ double sh[5][kLowRankBlock];
    const int tid = threadIdx.x;
    const int64_t t = (int64_t)blockIdx.x * kLowRankBlock + tid;
    double2 v = cz();
    if (t < count) {
        int p[R];
        if (R == 1) {
            p[0] = n;
        } else {
            int b[R];
            unrank_bars<R>((uint64_t)t, n, tab, b);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int lo = j == 0 ? -1 : b[j];
                const int hi = j == R - 1 ? n + R - 1 : b[j + 1];
                p[j] = hi - lo - 1;
            }
        }
        bool even = true;
        double w = 1.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            even = even && (p[j] % 2 == 0);
            for (int a = p[j] - 1; a > 1; a -= 2) w *= (double)a;
        }
        if (even) v = cscale(c[t], w);
    }
    sh[0][tid] = v.x;
    sh[1][tid] = 0.0;
    sh[2][tid] = v.y;
    sh[3][tid] = 0.0;
    sh[4][tid] = hypot(v.x, v.y);
    __syncthreads();
    for (int st = kLowRankBlock / 2; st > 0; st >>= 1) {
        if (tid < st) {
            const dd r = dd_add(dd{ sh[0][tid], sh[1][tid] }, dd{ sh[0][tid + st], sh[1][tid + st] });
            const dd i = dd_add(dd{ sh[2][tid], sh[3][tid] }, dd{ sh[2][tid + st], sh[3][tid + st] });
            sh[0][tid] = r.hi; sh[1][tid] = r.lo; sh[2][tid] = i.hi; sh[3][tid] = i.lo;
            sh[4][tid] += sh[4][tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        double* o = partials + 4 * (int64_t)blockIdx.x;
        o[0] = sh[0][0]; o[1] = sh[1][0]; o[2] = sh[2][0]; o[3] = sh[3][0];
        abs_partials[blockIdx.x] = sh[4][0];
    }
}

__global__ __launch_bounds__(256) void k_lowrank_abs_sum(const double* __restrict__ a, int64_t count,
                                                         double* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < count; k += 256) s += a[k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_lowrank_init(double2* c) { c[0] = cone(); }

static uint64_t binom_u(int a, int b) {
    if (b < 0 || b > a) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= b; ++i) r = r * (uint64_t)(a - b + i) / (uint64_t)i;
    return r;
}

template <int R>
static hipError_t lowrank_launches(const double2* dG, int ldg, int n, const uint64_t* tab, double2* c0, double2* c1,
                                   double* part, double* apart, double* asum, double* out_dd, hipStream_t st,
                                   int64_t* nslots) {
    hipLaunchKernelGGL(k_lowrank_init, dim3(1), dim3(1), 0, st, c0);
    double2* old_c = c0;
    double2* new_c = c1;
    for (int k = 1; k <= n; ++k) {
        const int64_t cnt = (int64_t)binom_u(k + R - 1, R - 1);
        hipLaunchKernelGGL(k_lowrank_step<R>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, dG, ldg, k, tab,
                           old_c, new_c, cnt);
        std::swap(old_c, new_c);
    }
    const int64_t cnt = (int64_t)binom_u(n + R - 1, R - 1);
    const int64_t blocks = (cnt + kLowRankBlock - 1) / kLowRankBlock;
    hipLaunchKernelGGL(k_lowrank_even_sum<R>, dim3((unsigned)blocks), dim3(kLowRankBlock), 0, st, old_c, n, tab, cnt,
                       part, apart);
    hipLaunchKernelGGL(k_lowrank_abs_sum, dim3(1), dim3(256), 0, st, apart, blocks, asum);
    *nslots = blocks;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(st, part, blocks, out_dd, nullptr, nullptr, 0);
}

}  // namespace hafgpu

using namespace hafgpu;

extern "C" int haf_lowrank_c128(const haf_cplx* G, int n, int r, int ldg, haf_cplx2* out, double* cond) {
    clear_error();
    if (!G || !out) return set_error(HAF_E_INVALID_ARG, "null pointer");
    if (n < 0 || r < 1 || (n > 0 && ldg < r))
        return set_error(HAF_E_INVALID_ARG, "bad n = %d / r = %d / ldg = %d", n, r, ldg);
    if (n > HAF_MAX_N) return set_error(HAF_E_TOO_LARGE, "n = %d exceeds the limit %d", n, HAF_MAX_N);
    if (r > kLowRankMaxR) return set_error(HAF_E_TOO_LARGE, "rank r = %d exceeds the limit %d", r, kLowRankMaxR);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < r; ++j) {
            const haf_cplx g = G[(int64_t)i * ldg + j];
            if (!std::isfinite(g.re) || !std::isfinite(g.im))
                return set_error(HAF_E_NONFINITE, "non-finite entry at (%d, %d)", i, j);
        }
    if (cond) *cond = 1.0;
    if (n == 0 || n % 2 == 1) {
        *out = haf_cplx2{ n == 0 ? 1.0 : 0.0, 0.0, 0.0, 0.0 };
        if (cond) *cond = n == 0 ? 1.0 : 0.0;
        return HAF_OK;
    }
    const int64_t mon = (int64_t)binom_u(n + r - 1, r - 1);
    if (mon > ((int64_t)1 << 28))
        return set_error(HAF_E_TOO_LARGE, "C(n + r - 1, r - 1) = %lld monomials exceed 2^28", (long long)mon);
    int rc = ensure_device(nullptr);
    if (rc) return rc;
    static thread_local hipStream_t st = nullptr;
    if (!st && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return set_error(HAF_E_DEVICE, "hipStreamCreate failed");
    Workspace* w = nullptr;
    if ((rc = workspace_for(st, &w))) return rc;
    const int64_t blocks = (mon + kLowRankBlock - 1) / kLowRankBlock;
    // coef: two coefficient vectors; part: double-double partials; aux: G, binomials, |.| partials, results
    const size_t g_b = ((size_t)n * r * sizeof(double2) + 255) & ~(size_t)255;
    const size_t tab_b = ((size_t)kBinA * kBinB * sizeof(uint64_t) + 255) & ~(size_t)255;
    const size_t abs_b = ((size_t)blocks * sizeof(double) + 255) & ~(size_t)255;
    if ((rc = workspace_reserve(w, st, 2 * (size_t)mon * sizeof(double2), (size_t)blocks * 4 * sizeof(double),
                                g_b + tab_b + abs_b + 256)))
        return rc;
    char* aux = (char*)w->aux;
    double2* dG = (double2*)aux;
    uint64_t* dtab = (uint64_t*)(aux + g_b);
    double* apart = (double*)(aux + g_b + tab_b);
    double* dres = (double*)(aux + g_b + tab_b + abs_b);      // 4 doubles result + 1 abs sum
    std::vector<uint64_t> tab((size_t)kBinA * kBinB);
    for (int a = 0; a < kBinA; ++a)
        for (int b = 0; b < kBinB; ++b) tab[(size_t)a * kBinB + b] = binom_u(a, b);
    std::vector<double2> hg((size_t)n * r);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < r; ++j) {
            const haf_cplx g = G[(int64_t)i * ldg + j];
            hg[(size_t)i * r + j] = make_double2(g.re, g.im);
        }
    if ((rc = hip_check(hipMemcpyAsync(dG, hg.data(), sizeof(double2) * hg.size(), hipMemcpyHostToDevice, st),
                        "factor upload")))
        return rc;
    if ((rc = hip_check(hipMemcpyAsync(dtab, tab.data(), sizeof(uint64_t) * tab.size(), hipMemcpyHostToDevice, st),
                        "binomial table upload")))
        return rc;
    double2* c0 = w->coef;
    double2* c1 = w->coef + mon;
    int64_t nslots = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (r) {
#define HAF_LR(RR) \
    case RR: e = lowrank_launches<RR>(dG, r, n, dtab, c0, c1, w->part, apart, dres + 4, dres, st, &nslots); break;
        HAF_LR(1) HAF_LR(2) HAF_LR(3) HAF_LR(4) HAF_LR(5) HAF_LR(6) HAF_LR(7) HAF_LR(8)
#undef HAF_LR
        default: break;
    }
    if ((rc = hip_check(e, "low-rank kernel launch"))) return rc;
    double h[5];
    if ((rc = hip_check(hipMemcpyAsync(h, dres, sizeof h, hipMemcpyDeviceToHost, st), "result download"))) return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "stream synchronize"))) return rc;
    *out = haf_cplx2{ h[0], h[1], h[2], h[3] };
    if (cond) {
        const double mag = std::hypot(h[0] + h[1], h[2] + h[3]);
        *cond = mag > 0.0 ? h[4] / mag : INFINITY;
    }
    return HAF_OK;
}
