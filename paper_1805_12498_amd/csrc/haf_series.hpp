// Series stage of one subset: from the coefficients a_k of det(I - lambda B)
// (and, for the loop hafnian, the loop moments l_k) to the term f(Z).
//   power traces   p_k = tr(B^k) = -k a_k - sum_{i<k} a_i p_{k-i}   (Newton's
//                  identities; App. B's route from the polynomial to the traces),
//   series         c_k = p_k / (2k) [+ l_k / 2],  f(Z) = [lambda^N] exp(sum_k c_k lambda^k)
//                  = e_N with e_0 = 1, e_j = (1/j) sum_{k=1}^{j} k c_k e_{j-k}
//                  (Eq. poly / Eq. haffinal: (1/N!) d^N/dlambda^N of the exponential
//                  series is its lambda^N coefficient).
// The arrays are sized by the compile-time bound NMAX and every loop is unrolled
// to it, so they stay in registers; the runtime N <= NMAX only guards the steps
// (uniform branches).  For a given N the operations and their order do not
// depend on NMAX, so every kernel that uses this gets bitwise the same f(Z).
#pragma once
#include "haf_common.hpp"

namespace hafgpu {

template <int NMAX, bool LOOPS>
__device__ __forceinline__ double2 subset_series_upto(const double2* __restrict__ coef, int64_t cstride, int t,
                                                      int N) {
    double2 a[NMAX + 1], p[NMAX + 1];
#pragma unroll
    for (int k = 1; k <= NMAX; ++k) a[k] = k <= N ? coef[(int64_t)(k - 1) * cstride + t] : cz();
    // Newton's identities
#pragma unroll
    for (int k = 1; k <= NMAX; ++k) {
        if (k <= N) {
            double2 acc = cscale(a[k], -(double)k);
#pragma unroll
            for (int i = 1; i < k; ++i) cfms(acc, a[i], p[k - i]);
            p[k] = acc;
        }
    }
    // k c_k = p_k / 2 [+ k l_k / 2]; kept in p
#pragma unroll
    for (int k = 1; k <= NMAX; ++k) {
        if (k <= N) {
            double2 kc = cscale(p[k], 0.5);
            if (LOOPS) {
                double2 l = coef[(int64_t)(N + k - 1) * cstride + t];
                kc.x = fma(0.5 * (double)k, l.x, kc.x);
                kc.y = fma(0.5 * (double)k, l.y, kc.y);
            }
            p[k] = kc;
        }
    }
    // exponential series, e_j in place of a_j (a is no longer needed)
    a[0] = cone();
    double2 res = a[0];
#pragma unroll
    for (int j = 1; j <= NMAX; ++j) {
        if (j <= N) {
            double2 acc = cz();
#pragma unroll
            for (int k = 1; k <= j; ++k) cfma(acc, p[k], a[j - k]);
            a[j] = cscale(acc, 1.0 / (double)j);
            res = a[j];
        }
    }
    return res;
}

}  // namespace hafgpu
