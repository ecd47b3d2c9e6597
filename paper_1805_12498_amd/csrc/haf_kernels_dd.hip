// Per-term double-double precision mode: the same per-subset route as the
// LDS-resident kernel (gather B = (X A_off) on Z, Eq. matA; loop moments;
// Householder reduction to Hessenberg form; characteristic polynomial of the
// Hessenberg form, App. B), then Newton's identities and the exponential
// series (Eq. poly, Eq. haffinal), every step in complex double-double.  The
// paper finds that the precision of each term, not the outer summation, sets
// the error of the alternating sum (Sec. 4.2) and suggests more precision for
// the terms; with about 106 bits per term the error of the sum drops from
// ~eps64 * kappa to ~eps_dd * kappa.  About ten to twenty times the work of the
// double path, so it is opt-in.
//
// Layout: one 64-lane workgroup per subset, the matrix in LDS as complex
// double-double (32 bytes per entry, odd pitch), s <= 64.  Coefficients go out
// as complex double-double (hi and lo parts in two planes); the series stage
// runs one lane per subset and adds the signed terms into double-double block
// partials in the slots the double path uses.
#include "haf_dd.hpp"
#include "haf_launch.hpp"

namespace hafgpu {

template <int SMAX, bool LOOPS>
__global__ __launch_bounds__(64) void k_coef_dd(const double2* __restrict__ A, int lda, int N, int m, uint64_t rank0,
                                                int count, const int* __restrict__ d_exp, double2* __restrict__ coef,
                                                int64_t cstride, int64_t lo_plane) {
    constexpr int P = SMAX + 1;
    __shared__ cdd H[SMAX * P];
    __shared__ cdd vec[SMAX];
    __shared__ int sidx[SMAX];
    const int lane = threadIdx.x;
    const int e = d_exp ? *d_exp : 0;
    const int s = 2 * m;
    // coefficient k of subset i: hi parts at coef[(k-1) cstride + i], lo parts lo_plane further
    auto store = [&](int k, int sub, cdd v) {
        coef[(int64_t)(k - 1) * cstride + sub] = make_double2(v.re.hi, v.im.hi);
        coef[lo_plane + (int64_t)(k - 1) * cstride + sub] = make_double2(v.re.lo, v.im.lo);
    };

    for (int sub = blockIdx.x; sub < count; sub += gridDim.x) {
        const uint32_t mask = unrank_subset(rank0 + (uint64_t)sub, m, N);
        __syncthreads();
        if (lane < s) sidx[lane] = subset_vertex(mask, lane);
        __syncthreads();
        // ---- gather (exact: a power-of-two scaling of double entries)
        if (lane < s) {
            const int col = sidx[lane];
            for (int r = 0; r < s; ++r)
                H[r * P + lane] = (lane == (r ^ 1)) ? cdd_zero()
                                                    : cdd_ldexp(cdd_of(A[(int64_t)(sidx[r] ^ 1) * lda + col]), -2 * e);
        }
        __syncthreads();
        // ---- loop moments l_k = d^T B^(k-1) (X d)
        if (LOOPS) {
            cdd d = cdd_zero(), y = cdd_zero();
            if (lane < s) {
                d = cdd_ldexp(cdd_of(A[(int64_t)sidx[lane] * lda + sidx[lane]]), -e);
                y = cdd_ldexp(cdd_of(A[(int64_t)sidx[lane ^ 1] * lda + sidx[lane ^ 1]]), -e);
            }
            for (int k = 1; k <= N; ++k) {
                const cdd t = cdd_mul(d, y);
                const cdd l = cdd{ dd_wave_sum(t.re), dd_wave_sum(t.im) };
                if (lane == 0) store(N + k, sub, l);
                if (k == N) break;
                if (lane < s) vec[lane] = y;
                __syncthreads();
                cdd acc = cdd_zero();
                if (lane < s)
                    for (int c = 0; c < s; ++c) acc = cdd_fma(acc, H[lane * P + c], vec[c]);
                y = acc;
                __syncthreads();
            }
        }
        // ---- Householder reduction to upper Hessenberg form
        for (int j = 0; j + 2 < s; ++j) {
            cdd x = cdd_zero();
            if (lane > j && lane < s) x = H[lane * P + j];
            // scale the column by an exact power of two of its largest entry
            double amax = fmax(fabs(x.re.hi), fabs(x.im.hi));
            for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
            if (amax < kTinyColumn) continue;
            const int sh = -ilogb(amax);
            x = cdd_ldexp(x, sh);
            dd sq = dd_of(0.0);
            if (lane >= j + 2) sq = dd_add(dd_mul(x.re, x.re), dd_mul(x.im, x.im));
            const dd sig = dd_wave_sum(sq);
            const cdd alpha = cdd_readlane(x, j + 1);
            if (dd_is_zero(sig) && dd_is_zero(alpha.im)) continue;
            const dd nrm = dd_sqrt(dd_add(dd_add(dd_mul(alpha.re, alpha.re), dd_mul(alpha.im, alpha.im)), sig));
            const dd beta = alpha.re.hi >= 0.0 ? dd_neg(nrm) : nrm;
            // P = I - tau v v^H with v_(j+1) = 1: tau = (beta - alpha) / beta, v_r = x_r / (alpha - beta)
            const cdd tau = cdd{ dd_div(dd_sub(beta, alpha.re), beta), dd_neg(dd_div(alpha.im, beta)) };
            const cdd scal = cdd_recip(cdd{ dd_sub(alpha.re, beta), alpha.im });
            if (lane < s) vec[lane] = lane == j + 1 ? cdd_one() : (lane > j + 1 ? cdd_mul(x, scal) : cdd_zero());
            __syncthreads();
            // left: H <- (I - conj(tau) v v^H) H on columns j+1..s-1
            if (lane > j && lane < s) {
                cdd w = cdd_zero();
                for (int r = j + 1; r < s; ++r) w = cdd_fma_cj(w, vec[r], H[r * P + lane]);
                const cdd wt = cdd_mul(cdd_conj(tau), w);
                for (int r = j + 1; r < s; ++r) H[r * P + lane] = cdd_fms(H[r * P + lane], vec[r], wt);
            }
            if (lane == j) H[(j + 1) * P + j] = cdd{ dd_ldexp(beta, -sh), dd_of(0.0) };
            __syncthreads();
            // right: H <- H (I - tau v v^H) on columns j+1..s-1, all rows
            if (lane < s) {
                cdd y = cdd_zero();
                for (int c = j + 1; c < s; ++c) y = cdd_fma(y, H[lane * P + c], vec[c]);
                const cdd yt = cdd_mul(y, tau);
                for (int c = j + 1; c < s; ++c) H[lane * P + c] = cdd_sub(H[lane * P + c], cdd_mul(yt, cdd_conj(vec[c])));
            }
            __syncthreads();
        }
        // ---- g_(r,c+1) = h_(r,c) prod_(k=r+1)^(c) h_(k,k-1), in place (lane = row)
        if (lane < s) {
            cdd pw = cdd_one();
            for (int c = lane; c < s; ++c) {
                H[lane * P + c] = cdd_mul(H[lane * P + c], pw);
                if (c + 1 < s) pw = cdd_mul(pw, H[(c + 1) * P + c]);
            }
        }
        __syncthreads();
        // ---- c_i(x) = det(x I - H[0:i, 0:i]) one degree at a time: lane i holds c_i[d]
        cdd prev = cdd_zero();
        for (int d = 0; d < s; ++d) {
            cdd shv;
            shv.re.hi = __shfl_up(prev.re.hi, 1, 64);
            shv.re.lo = __shfl_up(prev.re.lo, 1, 64);
            shv.im.hi = __shfl_up(prev.im.hi, 1, 64);
            shv.im.lo = __shfl_up(prev.im.lo, 1, 64);
            cdd acc = lane == 0 ? (d == 0 ? cdd_one() : cdd_zero()) : shv;
            cdd accs = cdd_readlane(prev, s - 1);
            for (int r = d; r < s; ++r) {                // c_r[d] = 0 for r < d
                const cdd b = cdd_readlane(acc, r);
                if (lane > r && lane < s) acc = cdd_fms(acc, H[r * P + lane - 1], b);
                accs = cdd_fms(accs, H[r * P + s - 1], b);
            }
            prev = acc;
            const int k = s - d;                         // coefficient of lambda^k in det(I - lambda B)
            if (k <= N && lane == 0) store(k, sub, accs);
        }
        if (lane == 0)
            for (int k = s + 1; k <= N; ++k) store(k, sub, cdd_zero());
    }
}

// One lane per subset: Newton's identities and the exponential series in
// complex double-double, then the signed double-double block sum (a fixed tree)
// into one partial slot (re_hi, re_lo, im_hi, im_lo).
template <bool LOOPS>
__global__ __launch_bounds__(256) void k_series_dd(const double2* __restrict__ coef, int64_t cstride,
                                                  int64_t lo_plane, int count, int N, double sign,
                                                  double* __restrict__ partials, int64_t slot0) {
    __shared__ double sh[4][256];
    const int t = blockIdx.x * 256 + threadIdx.x;
    cdd f = cdd_zero();
    if (t < count) {
        auto load = [&](int k) {
            const double2 h = coef[(int64_t)(k - 1) * cstride + t];
            const double2 l = coef[lo_plane + (int64_t)(k - 1) * cstride + t];
            return cdd{ dd{ h.x, l.x }, dd{ h.y, l.y } };
        };
        cdd a[33], p[33];
        for (int k = 1; k <= N; ++k) a[k] = load(k);
        for (int k = 1; k <= N; ++k) {                  // p_k = -k a_k - sum_(i<k) a_i p_(k-i)
            cdd acc = cdd_mul_dd(a[k], dd_of(-(double)k));
            for (int i = 1; i < k; ++i) acc = cdd_fms(acc, a[i], p[k - i]);
            p[k] = acc;
        }
        for (int k = 1; k <= N; ++k) {                  // k c_k = p_k / 2 [+ k l_k / 2]
            cdd kc = cdd_ldexp(p[k], -1);
            if (LOOPS) kc = cdd_add(kc, cdd_ldexp(cdd_mul_dd(load(N + k), dd_of((double)k)), -1));
            p[k] = kc;
        }
        a[0] = cdd_one();
        for (int j = 1; j <= N; ++j) {                  // e_j = (1/j) sum_k k c_k e_(j-k)
            cdd acc = cdd_zero();
            for (int k = 1; k <= j; ++k) acc = cdd_fma(acc, p[k], a[j - k]);
            const dd inv = dd_div(dd_of(1.0), dd_of((double)j));
            a[j] = cdd_mul_dd(acc, inv);
        }
        f = a[N];
    }
    const int tid = threadIdx.x;
    sh[0][tid] = sign * f.re.hi;
    sh[1][tid] = sign * f.re.lo;
    sh[2][tid] = sign * f.im.hi;
    sh[3][tid] = sign * f.im.lo;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            const dd r = dd_add(dd{ sh[0][tid], sh[1][tid] }, dd{ sh[0][tid + st], sh[1][tid + st] });
            const dd i = dd_add(dd{ sh[2][tid], sh[3][tid] }, dd{ sh[2][tid + st], sh[3][tid + st] });
            sh[0][tid] = r.hi; sh[1][tid] = r.lo; sh[2][tid] = i.hi; sh[3][tid] = i.lo;
        }
        __syncthreads();
    }
    if (tid == 0) {
        double* o = partials + 4 * (slot0 + blockIdx.x);
        o[0] = sh[0][0]; o[1] = sh[1][0]; o[2] = sh[2][0]; o[3] = sh[3][0];
    }
}

hipError_t launch_coef_dd(int s, bool loops, int grid, hipStream_t st, const double2* A, int lda, int N, int m,
                          uint64_t rank0, int count, const int* d_exp, double2* coef, int64_t cstride,
                          int64_t lo_plane) {
    if (count <= 0) return hipSuccess;
    if (grid > count) grid = count;
#define HAF_LAUNCH_DD(SM)                                                                                    \
    if (loops) hipLaunchKernelGGL((k_coef_dd<SM, true>), dim3(grid), dim3(64), 0, st, A, lda, N, m, rank0,   \
                                  count, d_exp, coef, cstride, lo_plane);                                   \
    else hipLaunchKernelGGL((k_coef_dd<SM, false>), dim3(grid), dim3(64), 0, st, A, lda, N, m, rank0, count, \
                            d_exp, coef, cstride, lo_plane);
    if (s <= 16) { HAF_LAUNCH_DD(16) }
    else if (s <= 32) { HAF_LAUNCH_DD(32) }
    else if (s <= 48) { HAF_LAUNCH_DD(48) }
    else if (s <= 64) { HAF_LAUNCH_DD(64) }
    else return hipErrorInvalidValue;
#undef HAF_LAUNCH_DD
    return hipGetLastError();
}

hipError_t launch_series_dd(bool loops, int count, int N, double sign, hipStream_t st, const double2* coef,
                            int64_t cstride, int64_t lo_plane, double* partials, int64_t slot0) {
    if (count <= 0) return hipSuccess;
    if (N < 1 || N > 32) return hipErrorInvalidValue;
    const int blocks = (count + 255) / 256;
    if (loops)
        hipLaunchKernelGGL(k_series_dd<true>, dim3(blocks), dim3(256), 0, st, coef, cstride, lo_plane, count, N, sign,
                           partials, slot0);
    else
        hipLaunchKernelGGL(k_series_dd<false>, dim3(blocks), dim3(256), 0, st, coef, cstride, lo_plane, count, N, sign,
                           partials, slot0);
    return hipGetLastError();
}

}  // namespace hafgpu
