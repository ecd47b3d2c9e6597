// Per-subset series and the signed compensated outer sum.
//
// Input: for each subset of one size class, the coefficients a_k of
// det(I - lambda B) (k = 1..N) and, for the loop hafnian, the loop moments l_k.
// Each thread owns one subset:
//   power traces   p_k = tr(B^k) = -k a_k - sum_{i<k} a_i p_{k-i}   (Newton's
//                  identities; App. B's route from the polynomial to the traces),
//   series         c_k = p_k / (2k) [+ l_k / 2],  f(Z) = [lambda^N] exp(sum_k c_k lambda^k)
//                  = e_N with e_0 = 1, e_j = (1/j) sum_{k=1}^{j} k c_k e_{j-k}
//                  (Eq. poly / Eq. haffinal: (1/N!) d^N/dlambda^N of the exponential
//                  series is its lambda^N coefficient),
//   signed sum     (-1)^(N-|Z|) f(Z) (Eq. Pset), accumulated in double-double by a
//                  fixed-shape tree in the block; one partial per block.
#include "haf_common.hpp"
#include "haf_launch.hpp"
#include "haf_series.hpp"

namespace hafgpu {

constexpr int kSeriesBlock = 256;

// Signed double-double sum of one term per thread by a fixed tree; thread 0
// stores (re_hi, re_lo, im_hi, im_lo) at out.
__device__ __forceinline__ void block_partial(double sign, double2 f, double* __restrict__ out) {
    __shared__ double sh[4][kSeriesBlock];
    const int tid = threadIdx.x;
    sh[0][tid] = sign * f.x;
    sh[1][tid] = 0.0;
    sh[2][tid] = sign * f.y;
    sh[3][tid] = 0.0;
    __syncthreads();
    for (int st = kSeriesBlock / 2; st > 0; st >>= 1) {
        if (tid < st) {
            dd r = dd_add(dd{ sh[0][tid], sh[1][tid] }, dd{ sh[0][tid + st], sh[1][tid + st] });
            dd i = dd_add(dd{ sh[2][tid], sh[3][tid] }, dd{ sh[2][tid + st], sh[3][tid + st] });
            sh[0][tid] = r.hi; sh[1][tid] = r.lo; sh[2][tid] = i.hi; sh[3][tid] = i.lo;
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = sh[0][0]; out[1] = sh[1][0]; out[2] = sh[2][0]; out[3] = sh[3][0];
    }
}

// One block = kSeriesBlock subsets.  If terms != nullptr the unsigned f(Z) are
// written out (no sum); otherwise the block's signed double-double partial goes
// to partials[4 * (slot0 + blockIdx.x) + {re_hi, re_lo, im_hi, im_lo}].
template <int N, bool LOOPS>
__global__ __launch_bounds__(kSeriesBlock) void k_series(const double2* __restrict__ coef, int64_t cstride,
                                                         int count, double sign, double* __restrict__ partials,
                                                         int64_t slot0, double2* __restrict__ terms,
                                                         const int* __restrict__ d_exp) {
    const int t = blockIdx.x * kSeriesBlock + threadIdx.x;
    double2 f = cz();
    if (t < count) f = subset_series_upto<N, LOOPS>(coef, cstride, t, N);
    if (terms) {
        // undo the input scaling: every term is homogeneous of degree N in B
        const int e2n = d_exp ? 2 * N * (*d_exp) : 0;
        if (t < count) terms[t] = make_double2(ldexp(f.x, e2n), ldexp(f.y, e2n));
        return;
    }
    block_partial(sign, f, partials + 4 * (slot0 + blockIdx.x));
}

// Matrices of a batch (every N <= NMAX): the workgroup finds its chunk by a
// binary search over the launch's chunk table, then as k_series with the
// chunk's own N (the series body gives bitwise the same term for a given N
// whatever its compile-time bound).
template <int NMAX, bool LOOPS>
__global__ __launch_bounds__(kSeriesBlock) void k_series_group(const GroupChunk* __restrict__ chunks, int nchunks,
                                                               const double2* __restrict__ coef,
                                                               double* __restrict__ partials) {
    const int blk = (int)blockIdx.x;
    int lo = 0, hi = nchunks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunks[mid].gstart <= blk) lo = mid;
        else hi = mid - 1;
    }
    const GroupChunk ch = chunks[lo];
    const int lb = blk - ch.gstart;
    const int t = lb * kSeriesBlock + threadIdx.x;
    double2 f = cz();
    if (t < ch.count) f = subset_series_upto<NMAX, LOOPS>(coef + ch.coff, ch.count, t, ch.N);
    block_partial(ch.sign, f, partials + 4 * (ch.slot + lb));
}

// Several chunks of one matrix (N <= 16): block b of chunk c covers the chunk's
// subsets b*kSeriesBlock.. and writes slot slot0[c] + b, as k_series would.
template <int N, bool LOOPS>
__global__ __launch_bounds__(kSeriesBlock) void k_series_multi(const double2* __restrict__ coef,
                                                               double* __restrict__ partials, MultiChunks mc) {
    int c = 0;
    while (c + 1 < mc.nc && (int)blockIdx.x >= mc.gstart[c + 1]) ++c;
    const int lb = (int)blockIdx.x - mc.gstart[c];
    const int t = lb * kSeriesBlock + threadIdx.x;
    const int count = mc.count[c];
    double2 f = cz();
    if (t < count) f = subset_series_upto<N, LOOPS>(coef + mc.coff[c], count, t, N);
    block_partial(mc.sign[c], f, partials + 4 * (mc.slot0[c] + lb));
}

#define HAF_INST_SERIES(NN)                                                                                    \
    template __global__ void k_series<NN, false>(const double2*, int64_t, int, double, double*, int64_t, double2*, \
                                                 const int*);                                                 \
    template __global__ void k_series<NN, true>(const double2*, int64_t, int, double, double*, int64_t, double2*,  \
                                                const int*);
HAF_INST_SERIES(1) HAF_INST_SERIES(2) HAF_INST_SERIES(3) HAF_INST_SERIES(4)
HAF_INST_SERIES(5) HAF_INST_SERIES(6) HAF_INST_SERIES(7) HAF_INST_SERIES(8)
HAF_INST_SERIES(9) HAF_INST_SERIES(10) HAF_INST_SERIES(11) HAF_INST_SERIES(12)
HAF_INST_SERIES(13) HAF_INST_SERIES(14) HAF_INST_SERIES(15) HAF_INST_SERIES(16)
HAF_INST_SERIES(17) HAF_INST_SERIES(18) HAF_INST_SERIES(19) HAF_INST_SERIES(20)
HAF_INST_SERIES(21) HAF_INST_SERIES(22) HAF_INST_SERIES(23) HAF_INST_SERIES(24)
HAF_INST_SERIES(25) HAF_INST_SERIES(26) HAF_INST_SERIES(27) HAF_INST_SERIES(28)
HAF_INST_SERIES(29) HAF_INST_SERIES(30) HAF_INST_SERIES(31) HAF_INST_SERIES(32)

using SeriesMultiFn = void (*)(const double2*, double*, MultiChunks);
#define HAF_SM(NN) { k_series_multi<NN, false>, k_series_multi<NN, true> },
static const SeriesMultiFn g_series_multi[17][2] = {
    { nullptr, nullptr },
    HAF_SM(1) HAF_SM(2) HAF_SM(3) HAF_SM(4) HAF_SM(5) HAF_SM(6) HAF_SM(7) HAF_SM(8)
    HAF_SM(9) HAF_SM(10) HAF_SM(11) HAF_SM(12) HAF_SM(13) HAF_SM(14) HAF_SM(15) HAF_SM(16)
};
#undef HAF_SM

int group_series_blocks(int count) { return (count + kSeriesBlock - 1) / kSeriesBlock; }

hipError_t launch_series_group(bool loops, int nmax, int blocks, hipStream_t st, const GroupChunk* chunks,
                               int nchunks, const double2* coef, double* partials) {
    if (nchunks < 1 || blocks < 1 || nmax < 1 || nmax > 32) return hipErrorInvalidValue;
    auto k = nmax <= 16 ? (loops ? k_series_group<16, true> : k_series_group<16, false>)
                        : (loops ? k_series_group<32, true> : k_series_group<32, false>);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(kSeriesBlock), 0, st, chunks, nchunks, coef, partials);
    return hipGetLastError();
}

hipError_t launch_series_multi(int N, bool loops, hipStream_t st, const double2* coef, double* partials,
                               MultiChunks mc) {
    if (N < 1 || N > 16 || mc.nc < 1 || mc.nc > kMultiMax) return hipErrorInvalidValue;
    int g = 0;
    for (int c = 0; c < mc.nc; ++c) {
        if (mc.count[c] <= 0) return hipErrorInvalidValue;
        mc.gstart[c] = g;
        g += (mc.count[c] + kSeriesBlock - 1) / kSeriesBlock;
    }
    mc.gstart[mc.nc] = g;
    hipLaunchKernelGGL(g_series_multi[N][loops ? 1 : 0], dim3(g), dim3(kSeriesBlock), 0, st, coef, partials, mc);
    return hipGetLastError();
}

// Fixed-order double-double sum of nslots partials (one block of 256 threads):
// thread t folds slots t, t+256, ... in order, then a fixed tree.  Writes the
// double-double result (if out_dd) and its rounding to complex double (if out).
__device__ __forceinline__ void reduce_partials_block(const double* __restrict__ partials, int64_t nslots,
                                                      double* __restrict__ out_dd, double2* __restrict__ out, int e,
                                                      int N) {
    __shared__ double sh[4][256];
    const int tid = threadIdx.x;
    dd r{ 0.0, 0.0 }, i{ 0.0, 0.0 };
    for (int64_t k = tid; k < nslots; k += 256) {
        const double* p = partials + 4 * k;
        r = dd_add(r, dd{ p[0], p[1] });
        i = dd_add(i, dd{ p[2], p[3] });
    }
    sh[0][tid] = r.hi; sh[1][tid] = r.lo; sh[2][tid] = i.hi; sh[3][tid] = i.lo;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            dd a = dd_add(dd{ sh[0][tid], sh[1][tid] }, dd{ sh[0][tid + st], sh[1][tid + st] });
            dd b = dd_add(dd{ sh[2][tid], sh[3][tid] }, dd{ sh[2][tid + st], sh[3][tid + st] });
            sh[0][tid] = a.hi; sh[1][tid] = a.lo; sh[2][tid] = b.hi; sh[3][tid] = b.lo;
        }
        __syncthreads();
    }
    if (tid == 0) {
        // undo the exact input scaling: haf(A) = 2^(2eN) haf(A')
        const int e2n = 2 * N * e;
        const double rh = ldexp(sh[0][0], e2n), rl = ldexp(sh[1][0], e2n);
        const double ih = ldexp(sh[2][0], e2n), il = ldexp(sh[3][0], e2n);
        if (out_dd) { out_dd[0] = rh; out_dd[1] = rl; out_dd[2] = ih; out_dd[3] = il; }
        if (out) *out = make_double2(rh + rl, ih + il);
    }
}

__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partials, int64_t nslots,
                                                          double* __restrict__ out_dd, double2* __restrict__ out,
                                                          const int* __restrict__ d_exp, int N) {
    reduce_partials_block(partials, nslots, out_dd, out, d_exp ? *d_exp : 0, N);
}

// One workgroup per matrix of a batch (the single-matrix reduction).
__global__ __launch_bounds__(256) void k_reduce_group(const GroupItem* __restrict__ items,
                                                       const double* __restrict__ partials) {
    const GroupItem it = items[blockIdx.x];
    if (it.cval != kGroupComputed) return;    // written by the prologue
    reduce_partials_block(partials + 4 * it.slot_base, it.nslots, it.out_dd, it.out, *it.exp, it.n / 2);
}

// Exponent of the exact input scaling.  With f the largest |Re|, |Im| of an
// off-diagonal entry, e = floor(ilogb(f) / 2): the off-diagonal part scaled by
// 2^-2e and the diagonal by 2^-e keep haf and lhaf exact up to the factor
// 2^(2eN) (the scaling laws of Sec. 2: haf(mu A) = mu^(n/2) haf(A) and
// lhaf(sqrt(mu) A_diag + mu A_off) = mu^(n/2) lhaf(A)).
__device__ __forceinline__ int prescale_exp_block(const double2* __restrict__ A, int n, int lda) {
    __shared__ double sh[256];
    double f = 0.0;
    for (int e = threadIdx.x; e < n * n; e += 256) {
        const int i = e / n, j = e % n;
        if (i != j) {
            const double2 v = A[(int64_t)i * lda + j];
            f = fmax(f, fmax(fabs(v.x), fabs(v.y)));
        }
    }
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    const double m = sh[0];
    int e = 0;
    if (m > 0.0 && m <= 1.7e308) e = ilogb(m) >> 1;   // arithmetic shift: floor for negatives too
    return e;
}

__global__ __launch_bounds__(256) void k_prescale(const double2* __restrict__ A, int n, int lda, int* __restrict__ d_exp) {
    const int e = prescale_exp_block(A, n, lda);
    if (threadIdx.x == 0) *d_exp = e;
}

// One workgroup per matrix of a batch: a constant result (n = 0, odd-n haf),
// or the dense padded copy of an odd-n loop hafnian (isolated vertex of loop
// weight 1, as the pad kernel builds it) and the exponent from the caller's
// matrix (padding adds only zeros off the diagonal, so the exponent is that of
// the padded matrix).
__global__ __launch_bounds__(256) void k_group_prologue(const GroupItem* __restrict__ items) {
    const GroupItem it = items[blockIdx.x];
    if (it.cval != kGroupComputed) {
        if (threadIdx.x == 0) {
            const double v = it.cval == kGroupConstOne ? 1.0 : 0.0;
            if (it.out) *it.out = make_double2(v, 0.0);
            if (it.out_dd) { it.out_dd[0] = v; it.out_dd[1] = 0.0; it.out_dd[2] = 0.0; it.out_dd[3] = 0.0; }
            *it.exp = 0;
        }
        return;
    }
    if (it.A != it.src) {
        double2* dst = const_cast<double2*>(it.A);
        for (int e = threadIdx.x; e < it.n * it.n; e += 256) {
            const int i = e / it.n, j = e % it.n;
            double2 v = cz();
            if (i < it.src_n && j < it.src_n) v = it.src[(int64_t)i * it.src_lda + j];
            else if (i == it.src_n && j == it.src_n) v = cone();
            dst[(int64_t)i * it.lda + j] = v;
        }
    }
    const int e = prescale_exp_block(it.src, it.src_n, it.src_lda);
    if (threadIdx.x == 0) *it.exp = e;
}

__global__ void k_scatter(const double2* __restrict__ in, const int* __restrict__ perm, int count,
                          double2* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[perm[i]] = in[i];
}

// Write a constant result (n = 0 gives 1, odd n gives 0 for haf).
__global__ void k_write_const(double re, double* __restrict__ out_dd, double2* __restrict__ out) {
    if (threadIdx.x == 0) {
        if (out_dd) { out_dd[0] = re; out_dd[1] = 0.0; out_dd[2] = 0.0; out_dd[3] = 0.0; }
        if (out) *out = make_double2(re, 0.0);
    }
}

// Copy an n x n matrix (leading dimension lda) into an (n+1) x (n+1) dense one
// with an isolated vertex whose loop weight is 1 (odd-n loop hafnian).
__global__ void k_pad_odd(const double2* __restrict__ A, int n, int lda, double2* __restrict__ out) {
    const int np = n + 1;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < np * np; e += gridDim.x * blockDim.x) {
        const int i = e / np, j = e % np;
        double2 v = cz();
        if (i < n && j < n) v = A[(int64_t)i * lda + j];
        else if (i == n && j == n) v = cone();
        out[e] = v;
    }
}

// The matrix of the complete bipartite graph K_{n,n} with edge weights W: its
// hafnian is perm(W) (the bipartite identity of Sec. 1.1).
__global__ void k_bipartite(const double2* __restrict__ W, int n, int ldw, double2* __restrict__ B) {
    const int m = 2 * n;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * m; e += gridDim.x * blockDim.x) {
        const int i = e / m, j = e % m;
        double2 v = cz();
        if (i < n && j >= n) v = W[(int64_t)i * ldw + (j - n)];
        else if (i >= n && j < n) v = W[(int64_t)j * ldw + (i - n)];
        B[e] = v;
    }
}

}  // namespace hafgpu

namespace hafgpu {

int series_block() { return kSeriesBlock; }

typedef void (*series_fn)(const double2*, int64_t, int, double, double*, int64_t, double2*, const int*);

#define HAF_SFN(NN) { k_series<NN, false>, k_series<NN, true> },
static const series_fn g_series[33][2] = {
    { nullptr, nullptr },
    HAF_SFN(1) HAF_SFN(2) HAF_SFN(3) HAF_SFN(4) HAF_SFN(5) HAF_SFN(6) HAF_SFN(7) HAF_SFN(8)
    HAF_SFN(9) HAF_SFN(10) HAF_SFN(11) HAF_SFN(12) HAF_SFN(13) HAF_SFN(14) HAF_SFN(15) HAF_SFN(16)
    HAF_SFN(17) HAF_SFN(18) HAF_SFN(19) HAF_SFN(20) HAF_SFN(21) HAF_SFN(22) HAF_SFN(23) HAF_SFN(24)
    HAF_SFN(25) HAF_SFN(26) HAF_SFN(27) HAF_SFN(28) HAF_SFN(29) HAF_SFN(30) HAF_SFN(31) HAF_SFN(32)
};
#undef HAF_SFN

hipError_t launch_series(int N, bool loops, int count, hipStream_t st, const double2* coef, int64_t cstride,
                         double sign, double* partials, int64_t slot0, double2* terms, const int* d_exp) {
    if (N < 1 || N > 32) return hipErrorInvalidValue;
    if (count <= 0) return hipSuccess;
    const int blocks = (count + kSeriesBlock - 1) / kSeriesBlock;
    hipLaunchKernelGGL(g_series[N][loops ? 1 : 0], dim3(blocks), dim3(kSeriesBlock), 0, st, coef, cstride, count,
                       sign, partials, slot0, terms, d_exp);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, const double* partials, int64_t nslots, double* out_dd, double2* out,
                         const int* d_exp, int N) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, st, partials, nslots, out_dd, out, d_exp, N);
    return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t st, const double2* in, const int* perm, int count, double2* out) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3((count + 255) / 256), dim3(256), 0, st, in, perm, count, out);
    return hipGetLastError();
}

hipError_t launch_prescale(hipStream_t st, const double2* A, int n, int lda, int* d_exp) {
    hipLaunchKernelGGL(k_prescale, dim3(1), dim3(256), 0, st, A, n, lda, d_exp);
    return hipGetLastError();
}

hipError_t launch_write_const(hipStream_t st, double re, double* out_dd, double2* out) {
    hipLaunchKernelGGL(k_write_const, dim3(1), dim3(64), 0, st, re, out_dd, out);
    return hipGetLastError();
}

hipError_t launch_group_prologue(hipStream_t st, const GroupItem* items, int nitems) {
    if (nitems < 1) return hipSuccess;
    hipLaunchKernelGGL(k_group_prologue, dim3(nitems), dim3(256), 0, st, items);
    return hipGetLastError();
}

hipError_t launch_reduce_group(hipStream_t st, const GroupItem* items, int nitems, const double* partials) {
    if (nitems < 1) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_group, dim3(nitems), dim3(256), 0, st, items, partials);
    return hipGetLastError();
}

hipError_t launch_bipartite(hipStream_t st, const double2* W, int n, int ldw, double2* B) {
    const int m = 2 * n;
    const int blocks = (m * m + 255) / 256;
    hipLaunchKernelGGL(k_bipartite, dim3(blocks), dim3(256), 0, st, W, n, ldw, B);
    return hipGetLastError();
}

hipError_t launch_pad_odd(hipStream_t st, const double2* A, int n, int lda, double2* out) {
    const int np = n + 1;
    const int blocks = (np * np + 255) / 256;
    hipLaunchKernelGGL(k_pad_odd, dim3(blocks), dim3(256), 0, st, A, n, lda, out);
    return hipGetLastError();
}

}  // namespace hafgpu
