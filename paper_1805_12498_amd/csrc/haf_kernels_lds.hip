// Per-subset stage, LDS-resident form: one 64-lane workgroup per subset Z.
//
// For each Z (a subset of m pairs, s = 2m rows) the workgroup
//   1. gathers B = (X A_off) restricted to Z   (Eq. matA: row r of B is row
//      idx[r]^1 of A, i.e. the partner vertex of the r-th vertex; A_off is A
//      with a zero diagonal);
//   2. for the loop hafnian, forms the loop moments l_k = d^T B^(k-1) (X d),
//      k = 1..N, d = diag(A) on Z (the loop term of the loop-hafnian formula,
//      Sec. 3.3, read through the loop-ended walks of Sec. 3.1);
//   3. reduces B to upper Hessenberg form H = Q^H B Q by Householder
//      reflectors (a similarity, so tr(H^k) = tr(B^k));
//   4. takes the characteristic polynomial of H by the recurrence over its
//      leading principal blocks (App. B: the power traces follow from it) and
//      writes a_k, k = 1..N, the coefficients of det(I - lambda B).
// The matrix lives in LDS (row-major, odd pitch), so any s <= 64 fits.
#include "haf_common.hpp"
#include "haf_launch.hpp"

namespace hafgpu {

template <int SMAX, bool LOOPS>
__global__ __launch_bounds__(64) void k_coef_lds(const double2* __restrict__ A, int lda, int N, int m,
                                                  uint64_t rank0, int count, const uint32_t* __restrict__ masks,
                                                  const int* __restrict__ d_exp, double2* __restrict__ coef,
                                                  int64_t cstride) {
    constexpr int P = SMAX + 1;                 // odd pitch
    __shared__ double2 H[SMAX * P];
    __shared__ double2 vec[SMAX];
    __shared__ int sidx[SMAX];
    const int lane = threadIdx.x;
    const int e = d_exp ? *d_exp : 0;
    const double off_scale = ldexp(1.0, -2 * e), diag_scale = ldexp(1.0, -e);

    for (int sub = blockIdx.x; sub < count; sub += gridDim.x) {
        const uint32_t mask = masks ? masks[sub] : unrank_subset(rank0 + (uint64_t)sub, m, N);
        const int s = 2 * __builtin_popcount(mask);
        if (s > SMAX || (N < 32 && (mask >> N) != 0u)) {   // mask outside the pairs: no term
            if (lane == 0)
                for (int k = 1; k <= (LOOPS ? 2 * N : N); ++k)
                    coef[(int64_t)(k - 1) * cstride + sub] = make_double2(__builtin_nan(""), __builtin_nan(""));
            continue;
        }
        __syncthreads();                        // previous subset is done with LDS
        if (lane < s) sidx[lane] = subset_vertex(mask, lane);
        __syncthreads();

        // ---- 1. gather: lane c fills column c
        if (lane < s) {
            const int col = sidx[lane];
            for (int r = 0; r < s; ++r) {
                const int row = sidx[r] ^ 1;
                H[r * P + lane] = (lane == (r ^ 1)) ? cz() : cscale(A[(int64_t)row * lda + col], off_scale);
            }
        }
        __syncthreads();

        // ---- 2. loop moments
        if (LOOPS) {
            double2 d = cz(), y = cz();
            if (lane < s) d = cscale(A[(int64_t)sidx[lane] * lda + sidx[lane]], diag_scale);
            y.x = __shfl_xor(d.x, 1, 64);       // (X d)_r = d_{r^1}
            y.y = __shfl_xor(d.y, 1, 64);
            for (int k = 1; k <= N; ++k) {
                double2 t = cmul(d, y);
                double lx = wave_sum(t.x), ly = wave_sum(t.y);
                if (lane == 0) coef[(int64_t)(N + k - 1) * cstride + sub] = make_double2(lx, ly);
                if (k == N) break;
                if (lane < s) vec[lane] = y;
                __syncthreads();
                double2 acc = cz();
                if (lane < s)
                    for (int c = 0; c < s; ++c) cfma(acc, H[lane * P + c], vec[c]);
                y = acc;
                __syncthreads();
            }
        }

        // ---- 3. Householder reduction to upper Hessenberg form
        for (int j = 0; j + 2 < s; ++j) {
            double2 x = cz();
            if (lane > j && lane < s) x = H[lane * P + j];
            // Work on the column scaled by an exact power of two of its largest entry, so a
            // column of rounding noise (low-rank B) cannot underflow |x|^2 into 0 or inf.
            const double amax = wave_max(fmax(fabs(x.x), fabs(x.y)));
            if (amax < kTinyColumn) continue;             // nothing below the diagonal to reduce
            const double sc = ldexp(1.0, -ilogb(amax));
            x = cscale(x, sc);
            const double sig = wave_sum(lane >= j + 2 ? fma(x.x, x.x, x.y * x.y) : 0.0);
            const double2 alpha = make_double2(readlane_d(x.x, j + 1), readlane_d(x.y, j + 1));
            if (sig == 0.0 && alpha.y == 0.0) continue;   // already reduced (uniform branch)
            const double nrm = sqrt(fma(alpha.x, alpha.x, fma(alpha.y, alpha.y, sig)));
            const double beta = alpha.x >= 0.0 ? -nrm : nrm;
            // P = I - tau v v^H with v_{j+1} = 1 satisfies P^H (alpha, x..) = (beta, 0..)
            const double2 tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
            const double2 scal = crecip(make_double2(alpha.x - beta, alpha.y));
            if (lane < s) vec[lane] = lane == j + 1 ? cone() : (lane > j + 1 ? cmul(x, scal) : cz());
            __syncthreads();
            // left: H <- (I - conj(tau) v v^H) H on columns j+1..s-1 (column j becomes beta e_{j+1})
            if (lane > j && lane < s) {
                double2 w = cz();
                for (int r = j + 1; r < s; ++r) cfma_cj(w, vec[r], H[r * P + lane]);
                const double2 wt = cmul(cconj(tau), w);
                for (int r = j + 1; r < s; ++r) cfms(H[r * P + lane], vec[r], wt);
            }
            if (lane == j) H[(j + 1) * P + j] = make_double2(beta / sc, 0.0);
            __syncthreads();
            // right: H <- H (I - tau v v^H) on columns j+1..s-1, all rows
            if (lane < s) {
                double2 y = cz();
                for (int c = j + 1; c < s; ++c) cfma(y, H[lane * P + c], vec[c]);
                const double2 yt = cmul(y, tau);
                for (int c = j + 1; c < s; ++c) cfms_cj(H[lane * P + c], yt, vec[c]);
            }
            __syncthreads();
        }

        // ---- 4a. scale the upper triangle: g_{r,i} = h_{r,i-1} prod_{k=r+1}^{i-1} h_{k,k-1},
        //          stored in place of h_{r,i-1}
        if (lane < s) {
            double2 pi = cone();
            for (int c = lane; c < s; ++c) {
                H[lane * P + c] = cmul(H[lane * P + c], pi);
                if (c + 1 < s) pi = cmul(pi, H[(c + 1) * P + c]);
            }
        }
        __syncthreads();

        // ---- 4b. characteristic polynomials c_i(x) = det(x I - H[0:i, 0:i]):
        //   c_i = x c_{i-1} - sum_{r<i} g_{r,i} c_r.   Solved one degree at a time:
        //   lane i holds c_i[d]; c_s is carried uniformly in every lane.
        double2 prev = cz();                    // c_i[d-1]
        for (int d = 0; d < s; ++d) {
            double2 sh;
            sh.x = __shfl_up(prev.x, 1, 64);
            sh.y = __shfl_up(prev.y, 1, 64);
            double2 acc = lane == 0 ? (d == 0 ? cone() : cz()) : sh;
            double2 accs = readlane_c(prev, s - 1);
            for (int r = d; r < s; ++r) {      // c_r[d] = 0 for r < d
                const double2 b = readlane_c(acc, r);
                if (lane > r && lane < s) cfms(acc, H[r * P + lane - 1], b);
                cfms(accs, H[r * P + s - 1], b);
            }
            prev = acc;
            const int k = s - d;                // coefficient of lambda^k in det(I - lambda B)
            if (k <= N && lane == 0) coef[(int64_t)(k - 1) * cstride + sub] = accs;
        }
        if (lane == 0)
            for (int k = s + 1; k <= N; ++k) coef[(int64_t)(k - 1) * cstride + sub] = cz();
    }
}

// Explicit instantiations (the host selects SMAX >= s).
#define HAF_INST_LDS(SM)                                                                                   \
    template __global__ void k_coef_lds<SM, false>(const double2*, int, int, int, uint64_t, int,            \
                                                   const uint32_t*, const int*, double2*, int64_t);         \
    template __global__ void k_coef_lds<SM, true>(const double2*, int, int, int, uint64_t, int,             \
                                                  const uint32_t*, const int*, double2*, int64_t);
HAF_INST_LDS(16)
HAF_INST_LDS(32)
HAF_INST_LDS(64)

}  // namespace hafgpu

namespace hafgpu {

hipError_t launch_coef_lds(int smax, bool loops, int grid, hipStream_t st, const double2* A, int lda, int N,
                           int m, uint64_t rank0, int count, const uint32_t* masks, const int* d_exp, double2* coef,
                           int64_t cstride) {
    if (count <= 0) return hipSuccess;
    if (grid > count) grid = count;
    dim3 g(grid), b(64);
#define HAF_LAUNCH_LDS(SM)                                                                                  \
    if (loops) hipLaunchKernelGGL((k_coef_lds<SM, true>), g, b, 0, st, A, lda, N, m, rank0, count, masks,   \
                                  d_exp, coef, cstride);                                                    \
    else hipLaunchKernelGGL((k_coef_lds<SM, false>), g, b, 0, st, A, lda, N, m, rank0, count, masks, d_exp, \
                            coef, cstride);
    if (smax <= 16) { HAF_LAUNCH_LDS(16) }
    else if (smax <= 32) { HAF_LAUNCH_LDS(32) }
    else if (smax <= 64) { HAF_LAUNCH_LDS(64) }
    else return hipErrorInvalidValue;
#undef HAF_LAUNCH_LDS
    return hipGetLastError();
}

}  // namespace hafgpu
