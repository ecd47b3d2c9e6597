// The subset sum over a prime field F_p, for exact hafnians and loop hafnians
// of integer matrices.
//
// Each term f(Z) of the sum (Sec. 3.2, Eq. Pset) counts the tangles of the
// cycle cover it belongs to, so it is an integer, and its route from B = X A_Z
// to f(Z) (Sec. 3.3 with the power traces of App. B) uses only field
// operations: a similarity to Hessenberg form, the characteristic polynomial
// of the Hessenberg form, Newton's identities (division by k <= n/2) and the
// exponential series (division by j <= n/2 and by 2).  Running the whole sum
// modulo a few primes p > n and combining the residues by Chinese remaindering
// gives the exact integer.
//
// Field elements are doubles holding integers in [0, p) with p < 2^25, so a
// product is exact (< 2^50), up to eight products can be added before a
// reduction (< 2^53), and x mod p is x - floor(x / p) p computed with one
// multiply by 1/p, a floor and an exact fused multiply-add, plus one
// correction either way (the quotient is off by at most one).
//
// Per subset (one 64-lane workgroup, matrix in LDS):
//   gather      B[r][c] = A[v(r)^1][v(c)] mod p, zero where c = r^1;
//   loop part   l_k = d^T B^(k-1) (X d) by k - 1 matrix-vector products;
//   Hessenberg  elimination without divisions: step j takes the pivot
//               h = B[j+1][j] (after exchanging in the first nonzero row of
//               column j below the diagonal, if needed), multiplies the rows
//               below it by h and subtracts B[r][j] times the pivot row, then
//               adds B[r][j] times column r to column j+1 after scaling it by h;
//               with the finished columns scaled by h too, this is h times a
//               similarity of the matrix.  The finished columns are never read
//               again by the elimination, so their scales are applied once at
//               the end (column k by the product of the pivots of the steps
//               after it).  The result is D H' with H' similar to B and D the
//               product of the pivots, so a_k(B) = a_k(D H') / D^k: one inverse
//               per subset;
//   polynomial  c_i = x c_(i-1) - sum_(r<i) g_(r,i) c_r over the leading blocks
//               of the Hessenberg form, g_(r,i) = h_(r,i-1) prod_(k=r+1)^(i-1)
//               h_(k,k-1), lanes over the degree.
// The series stage runs one lane per subset from the stored coefficients, and
// the signed terms are added per block of 256 subsets (exact in double, then
// reduced).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "haf_common.hpp"
#include "haf_modp.hpp"

namespace hafgpu {

struct Fp {
    double p, pinv;
};

// x mod p for an integer-valued double with |x| < 2^53
__device__ __forceinline__ double fp_red(const Fp& F, double x) {
    const double q = floor(x * F.pinv);
    double r = fma(-q, F.p, x);
    r = r < 0.0 ? r + F.p : r;
    return r >= F.p ? r - F.p : r;
}
__device__ __forceinline__ double fp_mul(const Fp& F, double a, double b) { return fp_red(F, a * b); }
__device__ __forceinline__ double fp_add(const Fp& F, double a, double b) {
    const double s = a + b;
    return s >= F.p ? s - F.p : s;
}
__device__ __forceinline__ double fp_sub(const Fp& F, double a, double b) {
    const double s = a - b;
    return s < 0.0 ? s + F.p : s;
}
// a^(p-2) = a^(-1) for a != 0 (Fermat), square-and-multiply from the top bit
__device__ __forceinline__ double fp_inv(const Fp& F, double a) {
    const uint32_t e = (uint32_t)F.p - 2u;
    double r = 1.0;
    for (int b = 31 - __builtin_clz(e); b >= 0; --b) {
        r = fp_mul(F, r, r);
        if ((e >> b) & 1u) r = fp_mul(F, r, a);
    }
    return r;
}

template <int SMAX, bool LOOPS>
__global__ __launch_bounds__(64) void k_modp_coef(const double* __restrict__ Ap, int n, int N, int m, uint64_t rank0,
                                                  int count, const ModpPrime* __restrict__ primes,
                                                  double* __restrict__ coef, int64_t cstride,
                                                  int64_t prime_stride) {
    constexpr int PITCH = SMAX + 1;
    constexpr int CT = (SMAX + 1) * (SMAX + 2) / 2;      // c_r[d] at r (r + 1) / 2 + d, d <= r
    __shared__ double H[SMAX * PITCH];
    __shared__ double ct[CT];
    __shared__ double vec[SMAX];                        // multipliers / loop vector
    __shared__ double hpiv[SMAX];                       // pivot of each step (1 where no step ran)
    __shared__ int sidx[SMAX];
    const int lane = threadIdx.x;
    const int pi = blockIdx.y;
    const Fp F{ primes[pi].p, primes[pi].pinv };
    const double* A = Ap + (int64_t)pi * n * n;
    double* cf = coef + (int64_t)pi * prime_stride;
    const int s = 2 * m;

    for (int sub = blockIdx.x; sub < count; sub += gridDim.x) {
        const uint32_t mask = unrank_subset(rank0 + (uint64_t)sub, m, N);
        __syncthreads();                                // the previous subset is done with LDS
        if (lane < s) sidx[lane] = subset_vertex(mask, lane);
        __syncthreads();
        // ---- gather: lane c fills column c
        if (lane < s) {
            const int col = sidx[lane];
            for (int r = 0; r < s; ++r) H[r * PITCH + lane] = (lane == (r ^ 1)) ? 0.0 : A[(sidx[r] ^ 1) * n + col];
        }
        __syncthreads();
        // ---- loop moments l_k = d^T B^(k-1) (X d)
        if (LOOPS) {
            double d = 0.0, y = 0.0;
            if (lane < s) {
                d = A[sidx[lane] * n + sidx[lane]];
                y = A[sidx[lane ^ 1] * n + sidx[lane ^ 1]];   // (X d)_r = d_(r^1)
            }
            for (int k = 1; k <= N; ++k) {
                // ell = sum_r d_r y_r: lane products, then a tree over the wave (each stage
                // adds two reduced values, < 2^26)
                double t = lane < s ? fp_mul(F, d, y) : 0.0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) t = fp_add(F, t, __shfl_xor(t, o, 64));
                if (lane == 0) cf[(int64_t)(N + k - 1) * cstride + sub] = t;
                if (k == N) break;
                if (lane < s) vec[lane] = y;
                __syncthreads();
                double acc = 0.0;
                if (lane < s) {
                    for (int c0 = 0; c0 < s; c0 += 8) {
                        double part = 0.0;
                        for (int c = c0; c < c0 + 8 && c < s; ++c) part = fma(H[lane * PITCH + c], vec[c], part);
                        acc = fp_add(F, acc, fp_red(F, part));
                    }
                }
                y = acc;
                __syncthreads();
            }
        }
        // ---- Hessenberg form by elimination without divisions
        if (lane < SMAX) hpiv[lane] = 1.0;
        for (int j = 0; j + 2 < s; ++j) {
            // first nonzero entry of column j below the diagonal
            const bool nz = lane > j && lane < s && H[lane * PITCH + j] != 0.0;
            const uint64_t hits = __ballot(nz);
            if (hits == 0) continue;                    // nothing to eliminate (uniform)
            const int pr = __builtin_ctzll(hits);
            if (pr != j + 1) {                          // exchange rows and columns pr and j + 1
                if (lane < s) {
                    const double t = H[pr * PITCH + lane];
                    H[pr * PITCH + lane] = H[(j + 1) * PITCH + lane];
                    H[(j + 1) * PITCH + lane] = t;
                }
                __syncthreads();
                if (lane < s) {
                    const double t = H[lane * PITCH + pr];
                    H[lane * PITCH + pr] = H[lane * PITCH + j + 1];
                    H[lane * PITCH + j + 1] = t;
                }
                __syncthreads();
            }
            const double h = H[(j + 1) * PITCH + j];
            if (lane == 0) hpiv[j] = h;
            // multipliers: c_r = B[r][j] for r > j + 1
            if (lane < s) vec[lane] = lane > j + 1 ? H[lane * PITCH + j] : 0.0;
            __syncthreads();
            // rows r > j + 1: h row_r - c_r row_(j+1), columns j + 1 .. s - 1 (lane = column)
            if (lane > j && lane < s) {
                const double pv = H[(j + 1) * PITCH + lane];
                for (int r = j + 2; r < s; ++r) {
                    const double t = vec[r] * pv;
                    H[r * PITCH + lane] = fp_red(F, fma(h, H[r * PITCH + lane], -t));
                }
            }
            __syncthreads();
            // column j + 1: h col_(j+1) + sum_(r > j+1) c_r col_r, every row (lane = row)
            if (lane < s) {
                double acc = fp_mul(F, h, H[lane * PITCH + j + 1]);
                for (int r0 = j + 2; r0 < s; r0 += 8) {
                    double part = 0.0;
                    for (int r = r0; r < r0 + 8 && r < s; ++r) part = fma(vec[r], H[lane * PITCH + r], part);
                    acc = fp_add(F, acc, fp_red(F, part));
                }
                H[lane * PITCH + j + 1] = acc;
            }
            __syncthreads();
        }
        // deferred scales of the finished columns: column k times the pivots of steps k .. s-3
        if (lane < s) {
            double sc = 1.0;
            for (int k = s - 3; k >= 0; --k) {
                sc = fp_mul(F, sc, hpiv[k]);
                if (lane <= k + 1) H[lane * PITCH + k] = fp_mul(F, H[lane * PITCH + k], sc);
            }
        }
        __syncthreads();
        // ---- polynomial stage: g_(r,c+1) = h_(r,c) prod_(k=r+1)^(c) h_(k,k-1), in place (lane = row)
        if (lane < s) {
            double pw = 1.0;
            for (int c = lane; c < s; ++c) {
                H[lane * PITCH + c] = fp_mul(F, H[lane * PITCH + c], pw);
                if (c + 1 < s) pw = fp_mul(F, pw, H[(c + 1) * PITCH + c]);
            }
        }
        if (lane == 0) ct[0] = 1.0;
        __syncthreads();
        // c_i[d] = c_(i-1)[d-1] - sum_(r=d)^(i-1) g_(r,i) c_r[d]   (lane = degree d)
        for (int i = 1; i <= s; ++i) {
            double v = 0.0;
            if (lane < i) {
                double acc = 0.0;
                for (int r0 = lane; r0 < i; r0 += 8) {
                    double part = 0.0;
                    for (int r = r0; r < r0 + 8 && r < i; ++r)
                        part = fma(H[r * PITCH + i - 1], ct[r * (r + 1) / 2 + lane], part);
                    acc = fp_add(F, acc, fp_red(F, part));
                }
                const double sh = lane > 0 ? ct[(i - 1) * i / 2 + lane - 1] : 0.0;
                v = fp_sub(F, sh, acc);
            }
            if (lane < i) ct[i * (i + 1) / 2 + lane] = v;
            if (lane == 0) ct[i * (i + 1) / 2 + i] = 1.0;
            __syncthreads();
        }
        // a_k(B) = [x^(s-k)] det(x I - D H') / D^k, D = product of the pivots
        double D = 1.0;
        for (int k = 0; k + 2 < s; ++k) D = fp_mul(F, D, hpiv[k]);
        const double Dinv = fp_inv(F, D);
        if (lane == 0) {
            double dk = 1.0;
            for (int k = 1; k <= N; ++k) {
                dk = fp_mul(F, dk, Dinv);
                const double a = k <= s ? fp_mul(F, ct[s * (s + 1) / 2 + (s - k)], dk) : 0.0;
                cf[(int64_t)(k - 1) * cstride + sub] = a;
            }
        }
    }
}

// One lane per subset: Newton's identities p_k = -k a_k - sum_(i<k) a_i p_(k-i),
// c_k = p_k / (2k) [+ l_k / 2], e_j = (1/j) sum_(k<=j) k c_k e_(j-k), f = e_N, then
// the signed block sum (-1)^(N-m) f over 256 subsets, reduced, into one slot.
template <bool LOOPS>
__global__ __launch_bounds__(256) void k_modp_series(const double* __restrict__ coef, int64_t cstride,
                                                     int64_t prime_stride, int count, int N, int negative,
                                                     const ModpPrime* __restrict__ primes,
                                                     double* __restrict__ partials, int64_t slot0,
                                                     int64_t slot_stride) {
    __shared__ double sh[256];
    const int pi = blockIdx.y;
    const ModpPrime& P = primes[pi];
    const Fp F{ P.p, P.pinv };
    const double* cf = coef + (int64_t)pi * prime_stride;
    const int t = blockIdx.x * 256 + threadIdx.x;
    double f = 0.0;
    if (t < count) {
        double a[kModpMaxN + 1], pk[kModpMaxN + 1];
        for (int k = 1; k <= N; ++k) a[k] = cf[(int64_t)(k - 1) * cstride + t];
        for (int k = 1; k <= N; ++k) {
            double acc = fp_mul(F, (double)k, a[k]);
            for (int i = 1; i < k; ++i) acc = fp_add(F, acc, fp_mul(F, a[i], pk[k - i]));
            pk[k] = acc == 0.0 ? 0.0 : F.p - acc;
        }
        // k c_k = p_k / 2 [+ k l_k / 2], kept in pk
        for (int k = 1; k <= N; ++k) {
            double kc = fp_mul(F, pk[k], P.inv[2]);
            if (LOOPS) kc = fp_add(F, kc, fp_mul(F, fp_mul(F, (double)k, cf[(int64_t)(N + k - 1) * cstride + t]), P.inv[2]));
            pk[k] = kc;
        }
        a[0] = 1.0;
        for (int j = 1; j <= N; ++j) {
            double acc = 0.0;
            for (int k = 1; k <= j; ++k) acc = fp_add(F, acc, fp_mul(F, pk[k], a[j - k]));
            a[j] = fp_mul(F, acc, P.inv[j]);
        }
        f = a[N];
        if (negative && f != 0.0) f = F.p - f;
    }
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {             // exact: 256 values < 2^25 add up below 2^33
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[(int64_t)pi * slot_stride + slot0 + blockIdx.x] = fp_red(F, sh[0]);
}

// One block per prime: the sum of its partial slots mod p.
__global__ __launch_bounds__(256) void k_modp_reduce(const double* __restrict__ partials, int64_t nslots,
                                                     int64_t slot_stride, const ModpPrime* __restrict__ primes,
                                                     double* __restrict__ residues) {
    __shared__ double sh[256];
    const int pi = blockIdx.x;
    const Fp F{ primes[pi].p, primes[pi].pinv };
    const double* p = partials + (int64_t)pi * slot_stride;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nslots; k += 256) acc = fp_add(F, acc, p[k]);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] = fp_add(F, sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) residues[pi] = sh[0];
}

hipError_t launch_modp_coef(int s, bool loops, int grid, int nprimes, hipStream_t st, const double* Ap, int n, int N,
                            int m, uint64_t rank0, int count, const ModpPrime* primes, double* coef, int64_t cstride,
                            int64_t prime_stride) {
    if (count <= 0) return hipSuccess;
    if (grid > count) grid = count;
    const dim3 g((unsigned)grid, (unsigned)nprimes), b(64);
#define HAF_LAUNCH_MODP(SM)                                                                                   \
    if (loops) hipLaunchKernelGGL((k_modp_coef<SM, true>), g, b, 0, st, Ap, n, N, m, rank0, count, primes, coef, \
                                  cstride, prime_stride);                                                        \
    else hipLaunchKernelGGL((k_modp_coef<SM, false>), g, b, 0, st, Ap, n, N, m, rank0, count, primes, coef,     \
                            cstride, prime_stride);
    if (s <= 16) { HAF_LAUNCH_MODP(16) }
    else if (s <= 32) { HAF_LAUNCH_MODP(32) }
    else if (s <= 48) { HAF_LAUNCH_MODP(48) }
    else if (s <= 64) { HAF_LAUNCH_MODP(64) }
    else return hipErrorInvalidValue;
#undef HAF_LAUNCH_MODP
    return hipGetLastError();
}

hipError_t launch_modp_series(bool loops, int count, int N, bool negative, int nprimes, hipStream_t st,
                              const double* coef, int64_t cstride, int64_t prime_stride, const ModpPrime* primes,
                              double* partials, int64_t slot0, int64_t slot_stride) {
    if (count <= 0) return hipSuccess;
    if (N < 1 || N > kModpMaxN) return hipErrorInvalidValue;
    const dim3 g((unsigned)((count + 255) / 256), (unsigned)nprimes), b(256);
    if (loops)
        hipLaunchKernelGGL(k_modp_series<true>, g, b, 0, st, coef, cstride, prime_stride, count, N, negative ? 1 : 0,
                           primes, partials, slot0, slot_stride);
    else
        hipLaunchKernelGGL(k_modp_series<false>, g, b, 0, st, coef, cstride, prime_stride, count, N, negative ? 1 : 0,
                           primes, partials, slot0, slot_stride);
    return hipGetLastError();
}

hipError_t launch_modp_reduce(int nprimes, hipStream_t st, const double* partials, int64_t nslots,
                              int64_t slot_stride, const ModpPrime* primes, double* residues) {
    hipLaunchKernelGGL(k_modp_reduce, dim3((unsigned)nprimes), dim3(256), 0, st, partials, nslots, slot_stride, primes,
                       residues);
    return hipGetLastError();
}

}  // namespace hafgpu
