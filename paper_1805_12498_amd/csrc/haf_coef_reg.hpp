// Per-subset stage, register-tiled form (the hot path for subsets of s <= 48 rows).
//
// Same mathematics as the LDS-resident kernel (gather B = (X A_off) on Z, loop
// moments, Householder reduction to Hessenberg form, characteristic polynomial
// of the Hessenberg form; App. B and Sec. 3.3), laid out for 64-lane CDNA
// wavefronts:
//
//  * a group of L = P*Q lanes owns one subset matrix; a wave holds W = 64/L groups
//    (one size class per launch, so every group has the same s);
//  * lane (a, b) of a group keeps the R x C tile of B with rows a + P t and
//    columns b + Q u in VGPRs (2D cyclic distribution, so every lane keeps work as
//    the active trailing block of the reduction shrinks);
//  * the reduction step index j is a runtime loop; tile slots are static and
//    column slots left of the active block are skipped with uniform branches, so
//    nothing is indexed dynamically in registers (some layouts also drop, per
//    phase of the loop, the left-update terms of row slots above the reflector);
//  * one reduction step is one pass over the tile: with P = I - tau v v^H,
//        P^H H P = H - v w'^T - y1 v^H,   w' = conj(tau) (v^H H)^T,
//        y1 = tau (H v - conj(tau) gamma v),  gamma = v^H H v,
//    so both dot products come from the same tile and one update follows;
//  * every cross-lane exchange of a vector goes through LDS as a transposition:
//    lanes write per-tile partial sums, the lane that owns index i adds its P (or
//    Q) partials, and the result is read back by the lanes that need it.  On
//    gfx950 a 16-byte LDS read costs about one FP64 FMA, far less than moving the
//    same bytes with DPP, swizzle or readlane;
//  * the column norm each reflector needs comes from the column's owners: when
//    they broadcast the column they also store the sum of |h|^2 over their rows,
//    and every lane adds the P row-group values in the same fixed order;
//  * the wave raises its issue priority over the serial parts of a step (the
//    reflector, the partial sums, the broadcasts) and lowers it over the FMA
//    passes, so that the other wave on the SIMD keeps the FMA pipe busy;
//  * the characteristic polynomial is built with lanes over the degree d and the
//    polynomials c_r in registers, fully unrolled for the exact s (so register
//    slots and LDS offsets are static); the scaled Hessenberg entries g_{r,i} come
//    from LDS, one read per complex multiply-add.
//
// The per-subset body lives in this header so that the one-size-class kernel,
// the multi-chunk kernel and the shared batched / serving stage kernel run exactly
// the same arithmetic.
#pragma once
#include <type_traits>
#include <utility>

#include "haf_common.hpp"

namespace hafgpu {


// f(std::integral_constant<int, 0>{}), ..., f(std::integral_constant<int, N - 1>{})
template <int... I, class F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, I...>, F&& f) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

template <int P, int Q, int R, int C>
struct RegShape {
    static constexpr int L = P * Q;                        // lanes per matrix
    static constexpr int W = 64 / L;                       // matrices per wave
    static constexpr int SM = (P * R < Q * C) ? P * R : Q * C;   // largest s
    // transposition area: the w partial of column c from row group a sits at
    // c + WA * a, the y partial of row r from column group b at r + YB * b.  The pads
    // make both the stores (lane = (a, b)) and the sums (lane = column or row) hit
    // distinct LDS banks in every run of 8 or 16 lanes.
    static constexpr int WA = Q * C + ((C % 2 == 0) ? Q : 0);
    static constexpr int YB = P * R + (Q >= 8 ? 1 : 2);
    static constexpr int RED = P * WA + Q * YB;
    static constexpr int VEC = 4 * SM + SM / 2;            // column, v, w', y1, row-group norms
    static constexpr int GN = SM * (SM + 1) / 2;           // packed upper triangle
    static constexpr int SLACK = 8 * W;                    // zeroed, read past the table in whole chunks
    // during the reduction the area holds the partials and the vectors; afterwards
    // the packed table (+ slack) overwrites both
    static constexpr int AREA = RED + VEC > GN + SLACK ? RED + VEC : GN + SLACK;
    static constexpr int PER = AREA + SM;                  // + subdiagonal
    static constexpr int NI = (SM + L - 1) / L;            // vector indices per lane: lam, lam + L
    static_assert(L * W == 64, "group size must divide 64");
    static_assert(NI <= 2, "at most two vector indices per lane");
    static_assert((P & (P - 1)) == 0 && (Q & (Q - 1)) == 0 && P <= SM, "tree sums over P and Q; P norms fit the spare");
};

// Sum of K values at p[0], p[D], ..., p[(K-1) D] by a fixed pairwise tree
// (K a power of two): the same rounding as any lane doing the same sum, and a
// dependency chain of log2 K additions instead of K.
template <int K, int D>
__device__ __forceinline__ double2 tree_sum(const double2* __restrict__ p) {
    if constexpr (K == 1) {
        return p[0];
    } else {
        const double2 l = tree_sum<K / 2, D>(p), r = tree_sum<K / 2, D>(p + (K / 2) * D);
        return make_double2(l.x + r.x, l.y + r.y);
    }
}

template <int K>
__device__ __forceinline__ double tree_sum_d(const double* __restrict__ p) {
    if constexpr (K == 1) return p[0];
    else return tree_sum_d<K / 2>(p) + tree_sum_d<K / 2>(p + K / 2);
}

// Next subset of the same size in increasing mask order (= the next rank of the
// combinatorial number system), by Gosper's bit trick.
__device__ __forceinline__ uint32_t next_subset(uint32_t x) {
    const uint32_t r = x + (x & (0u - x));
    return (((r ^ x) >> 2) >> __builtin_ctz(x)) | r;
}

// Mask of the q-th subset of a run starting at rank `first` (in masks[], or by
// unranking rank0 + first and Gosper steps from `prev`); past the end of the
// chunk any m-subset stands in (computed, never written).
__device__ __forceinline__ uint32_t run_subset_mask(int q, uint32_t prev, int first, int count,
                                                    const uint32_t* __restrict__ masks, uint64_t rank0, int m, int N) {
    const int sub = first + q;
    const bool valid = sub < count;
    uint32_t mk;
    if (masks) mk = masks[valid ? sub : 0];
    else mk = q == 0 ? unrank_subset(rank0 + (uint64_t)(valid ? sub : 0), m, N) : next_subset(prev);
    return valid ? mk : (1u << m) - 1u;
}

// Lane (a, b)'s tile of B = X A_off on the subset: row r of B is row v(r)^1 of
// A and column c is column v(c), v(r) = member r&1 of the (r/2)-th chosen pair.
// The lane's rows a + P t are found by stepping over P/2 pairs at a time (P and
// Q are even, so the member bit is a&1 for all of them; likewise for columns).
template <int P, int Q, int R, int C>
__device__ __forceinline__ void gather_tile(double2 (&hh)[R][C], uint32_t mk, int a, int b, int s,
                                            const double2* __restrict__ A, int lda, double off_scale) {
    int rv[R], cv[C];
    uint32_t mm = mk;
    for (int z = 0; z < (a >> 1); ++z) mm &= mm - 1u;
#pragma unroll
    for (int t = 0; t < R; ++t) {
        rv[t] = (a + P * t < s) ? 2 * __builtin_ctz(mm) + (a & 1) : 0;
#pragma unroll
        for (int z = 0; z < P / 2; ++z) mm &= mm - 1u;
    }
    mm = mk;
    for (int z = 0; z < (b >> 1); ++z) mm &= mm - 1u;
#pragma unroll
    for (int u = 0; u < C; ++u) {
        cv[u] = (b + Q * u < s) ? 2 * __builtin_ctz(mm) + (b & 1) : 0;
#pragma unroll
        for (int z = 0; z < Q / 2; ++z) mm &= mm - 1u;
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const double2* arow = A + (int64_t)(rv[t] ^ 1) * lda;
#pragma unroll
        for (int u = 0; u < C; ++u) {
            const int r = a + P * t, c = b + Q * u;
            hh[t][u] = (r < s && c < s && c != (r ^ 1)) ? cscale(arow[cv[u]], off_scale) : cz();
        }
    }
}

// Characteristic polynomials of the leading principal blocks of the Hessenberg
// form, c_i(x) = det(x I - H[0:i, 0:i]), by c_i = x c_{i-1} - sum_{r<i} g_{r,i} c_r
// with the pre-scaled entries g_{r,i} = h_{r,i-1} prod_{k=r+1}^{i-1} h_{k,k-1} in a
// packed table gt (column i-1 holds rows 0..i-1).  A lane holds the degree-d
// coefficients c_r[d] of the rows r = h (mod SPLIT) in registers; the SPLIT lanes
// with the same d sit at lane distance 64/SPLIT and add their partial sums.  Rows
// below R0 are known to be zero at the degrees this call covers (the second pass
// of the degree split), so their slots are skipped.  The shift c_{i-1}[d-1] comes
// from the neighbouring lane, or from `bin` (c_{i-1}[d0-1], written by the first
// pass) for the lowest degree d0 of the call; `bout`, if given, receives
// c_i[d_top] for every i.  Each step reads its column in chunks of 8 (the table is
// followed by zeroed slack, so whole chunks are safe), the first chunk one step
// ahead, and keeps the FMA pipeline fed with two accumulators.
template <int S, int SPLIT, int R0>
__device__ __forceinline__ double2 charpoly_lanes(const double2* __restrict__ gt, int d, int h, int dlo,
                                                  const double2* __restrict__ bin, double2* __restrict__ bout,
                                                  int dtop) {
    constexpr int K = (S - R0 + SPLIT - 1) / SPLIT;     // register slots per lane
    double2 cr[K > 0 ? K : 1];
#pragma unroll
    for (int k = 0; k < K; ++k) cr[k] = cz();
    // rows r = R0 + k*SPLIT + h; c_{R0}... start from c_i = 0 at these degrees, except c_0 = 1
    if (R0 == 0 && h == 0 && d == 0) cr[0] = cone();
    double2 prev = (R0 == 0 && d == 0) ? cone() : cz();
    constexpr int I0 = R0 > 0 ? R0 : 1;
    // the first chunk of each step's column is read one step ahead, so its LDS latency
    // overlaps the previous step's multiply-adds and reduction (the table is read-only here)
    double2 gnext[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (k < K) gnext[k] = gt[(I0 - 1) * I0 / 2 + R0 + k * SPLIT + h];
#pragma unroll
    for (int i = I0; i <= S; ++i) {
        const int nk = (i - R0 + SPLIT - 1) / SPLIT;    // slots that may hold r < i (compile-time)
        double2 gcur[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) gcur[k] = gnext[k];
        if (i < S) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k < K) gnext[k] = gt[i * (i + 1) / 2 + R0 + k * SPLIT + h];
        }
        double2 acc[2] = { cz(), cz() };
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < K && k < nk) cfma(acc[k & 1], gcur[k], cr[k]);
#pragma unroll
        for (int c0 = 8; c0 < nk; c0 += 8) {
            double2 gv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (c0 + k < K) gv[k] = gt[(i - 1) * i / 2 + R0 + (c0 + k) * SPLIT + h];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (c0 + k < K) cfma(acc[k & 1], gv[k], cr[c0 + k]);
        }
        __builtin_amdgcn_s_setprio(2);        // the reduction and shift form the serial chain
        double2 tot = cadd(acc[0], acc[1]);
        if (SPLIT >= 4) { tot.x += swizzle_d<0x401F>(tot.x); tot.y += swizzle_d<0x401F>(tot.y); }   // lane ^ 16
        if (SPLIT >= 2) { tot.x = halves_sum(tot.x); tot.y = halves_sum(tot.y); }               // + lane ^ 32
        double2 sh;
        sh.x = dpp_d<0x138>(prev.x);          // wave_shr:1 -> c_{i-1}[d-1]
        sh.y = dpp_d<0x138>(prev.y);
        if (d == dlo) sh = bin ? bin[i - 1] : cz();
        const double2 ci = csub(sh, tot);
        if (i < S) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k == (i - R0) / SPLIT && h == (i - R0) % SPLIT) cr[k] = ci;
        }
        if (bout && i < S && d == dtop && h == 0) bout[i] = ci;   // bout has S entries
        prev = ci;
        __builtin_amdgcn_s_setprio(0);
        // the step's other reads stay within it: hoisting them further ahead only raises
        // register pressure (and occupancy is what hides their latency)
        __builtin_amdgcn_sched_barrier(0);
    }
    return prev;
}

#define HAF_CP_CASES                                                                                         \
    HAF_CP_CASE(2) HAF_CP_CASE(4) HAF_CP_CASE(6) HAF_CP_CASE(8) HAF_CP_CASE(10) HAF_CP_CASE(12)             \
    HAF_CP_CASE(14) HAF_CP_CASE(16) HAF_CP_CASE(18) HAF_CP_CASE(20) HAF_CP_CASE(22) HAF_CP_CASE(24)         \
    HAF_CP_CASE(26) HAF_CP_CASE(28) HAF_CP_CASE(30) HAF_CP_CASE(32) HAF_CP_CASE(34) HAF_CP_CASE(36)         \
    HAF_CP_CASE(38) HAF_CP_CASE(40) HAF_CP_CASE(42) HAF_CP_CASE(44) HAF_CP_CASE(46) HAF_CP_CASE(48)

// Each lane writes 16 B of a different line and a line fills over several subsets of
// its group.  With NTS the stores are nontemporal: launches over one large chunk then
// leave about a third less HBM write traffic at the same speed.  The batched and
// server stages, whose series launch reads the coefficients back at once, keep
// ordinary stores (nontemporal ones made the batched call 0.4% slower).
template <bool NTS>
__device__ __forceinline__ void store_coef(double2* p, double2 v) {
    if constexpr (NTS) {
        typedef double v2d __attribute__((ext_vector_type(2)));
        const v2d x = { v.x, v.y };
        __builtin_nontemporal_store(x, reinterpret_cast<v2d*>(p));
    } else {
        *p = v;
    }
}

// a_k = c_s[s-k], the lambda^k coefficient of det(I - lambda B), from lane d, plus
// zeros for s < k <= N
template <bool NTS>
__device__ __forceinline__ void write_coefs(double2* __restrict__ coef, int64_t cstride, bool valid, int sub, int s,
                                            int N, int d, int L, double2 cs) {
    if (!valid) return;
    const int k = s - d;
    if (d < s && k <= N) store_coef<NTS>(&coef[(int64_t)(k - 1) * cstride + sub], cs);
    for (int kk = s + 1 + d; kk <= N; kk += L) store_coef<NTS>(&coef[(int64_t)(kk - 1) * cstride + sub], cz());
}
template <bool NTS>
__device__ __forceinline__ void write_coefs_range(double2* __restrict__ coef, int64_t cstride, bool valid, int sub,
                                                  int s, int N, int d, int dlo, int dhi, double2 cs) {
    if (!valid || d < dlo || d >= dhi || d >= s) return;
    const int k = s - d;
    if (k <= N) store_coef<NTS>(&coef[(int64_t)(k - 1) * cstride + sub], cs);
}

// CP selects how the polynomial stage uses the wave: 0 = every group on its own
// matrix, 1 = the whole wave on one matrix at a time with the rows split over the
// W lane groups, 2 = one matrix per wave, degrees in two passes (below 32 with the
// rows split over the two lane halves, then the rest), 3 = the groups in pairs,
// each 32-lane half of the wave over the degrees of one matrix (for groups of
// fewer lanes than the matrix has rows).
//
// Vector stages give lane lam of a group the indices lam and, when the matrix
// has more rows than the group has lanes, lam + L.
template <int P, int Q, int R, int C, int CP, bool LOOPS, bool NTS = true>
__device__ __forceinline__ void coef_reg_span(double2* __restrict__ lds, const double2* __restrict__ A, int lda,
                                              int N, int m, uint64_t rank0, int count,
                                              const uint32_t* __restrict__ masks, double off_scale,
                                              double diag_scale, double2* __restrict__ coef, int64_t cstride,
                                              int grp0, int span, int tid) {
    using S = RegShape<P, Q, R, C>;
    constexpr int L = S::L, W = S::W, SM = S::SM, NI = S::NI;
    static_assert(CP == 3 ? (W % 2 == 0 && SM <= 32) : SM <= L, "the polynomial stage needs one lane per degree");

    const int g = tid / L;                    // group (matrix) in the wave
    const int lam = tid % L;                  // lane in the group
    const int a = lam / Q, b = lam % Q;       // row group, column group
    double2* red = lds + g * S::PER;          // transposition area / packed polynomial table
    double2* colb = red + S::RED;             // column j of H
    double2* vv = colb + SM;                  // Householder vector v
    double2* wb = vv + SM;                    // w' = conj(tau) v^H H
    double2* yb = wb + SM;                    // y1 = tau (H v - conj(tau) gamma v)
    double* nrmp = (double*)(yb + SM);        // per row group: squared norm of the next column below its subdiagonal
    double2* beta = red + S::AREA;            // subdiagonal of the Hessenberg form
    double2* wpart = red;                     // [a][column], row stride WA
    double2* ypart = red + P * S::WA;         // [b][row], stride YB
    const int s = 2 * m;

    // tid = lane in the wave; group g of the wave owns the run of `span` subsets starting at (grp0 + g) * span
    const int first = (grp0 + g) * span;
    uint32_t mask = 0;
    for (int q = 0; q < span; ++q) {
        const int sub = first + q;
        const bool valid = sub < count;
        mask = run_subset_mask(q, mask, first, count, masks, rank0, m, N);
        double2 h[R][C];
        gather_tile<P, Q, R, C>(h, mask, a, b, s, A, lda, off_scale);

        // ---- loop moments l_k = d^T B^(k-1) X d  (lane lam owns index lam of d)
        if (LOOPS) {
            double2 dl[NI], dp[NI];
#pragma unroll
            for (int z = 0; z < NI; ++z) {
                const int i = lam + z * L;
                const int vl = i < s ? subset_vertex(mask, i) : 0;
                dl[z] = i < s ? cscale(A[(int64_t)vl * lda + vl], diag_scale) : cz();
                dp[z] = i < s ? cscale(A[(int64_t)(vl ^ 1) * lda + (vl ^ 1)], diag_scale) : cz();
            }
            double2 yc[C];                     // y at own columns; y_0 = X d, (X d)_c = d_{c^1}
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const int vc = (b + Q * u < s) ? subset_vertex(mask, b + Q * u) ^ 1 : 0;
                yc[u] = (b + Q * u < s) ? cscale(A[(int64_t)vc * lda + vc], diag_scale) : cz();
            }
            double2 prod = cmul(dl[0], dp[0]);
#pragma unroll
            for (int z = 1; z < NI; ++z) prod = cadd(prod, cmul(dl[z], dp[z]));
            double lx = group_sum<L>(prod.x), ly = group_sum<L>(prod.y);
            if (valid && lam == 0) store_coef<NTS>(&coef[(int64_t)N * cstride + sub], make_double2(lx, ly));
            for (int k = 2; k <= N; ++k) {
                __builtin_amdgcn_s_setprio(0);
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    double2 acc = cz();
#pragma unroll
                    for (int u = 0; u < C; ++u) cfma(acc, h[t][u], yc[u]);
                    ypart[a + P * t + S::YB * b] = acc;
                }
                __builtin_amdgcn_s_setprio(2);    // sums, moment and broadcast: the serial part
                __syncthreads();
                double2 yr[NI];               // (B y) at the lane's indices
#pragma unroll
                for (int z = 0; z < NI; ++z) {
                    const int i = lam + z * L;
                    yr[z] = i < s ? tree_sum<Q, S::YB>(ypart + i) : cz();
                }
                prod = cmul(dl[0], yr[0]);
#pragma unroll
                for (int z = 1; z < NI; ++z) prod = cadd(prod, cmul(dl[z], yr[z]));
                lx = group_sum<L>(prod.x);
                ly = group_sum<L>(prod.y);
                if (valid && lam == 0) store_coef<NTS>(&coef[(int64_t)(N + k - 1) * cstride + sub], make_double2(lx, ly));
                if (k == N) break;
#pragma unroll
                for (int z = 0; z < NI; ++z)
                    if (lam + z * L < SM) yb[lam + z * L] = yr[z];
                __syncthreads();
#pragma unroll
                for (int u = 0; u < C; ++u) yc[u] = (b + Q * u < s) ? yb[b + Q * u] : cz();
            }
            __builtin_amdgcn_s_setprio(0);
        }

        // ---- Householder reduction to upper Hessenberg form
        if (b == 0) {                          // column 0 -> colb, its norm below row 1 -> nrmp
            double part = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if (a + P * t < SM) colb[a + P * t] = h[t][0];
                if (a + P * t >= 2) part = fma(h[t][0].x, h[t][0].x, fma(h[t][0].y, h[t][0].y, part));
            }
            nrmp[a] = part;
        }
        // one Householder step; row slots below TLO hold only rows <= j, where v = 0,
        // so the left-update terms of those slots are left out at compile time
        auto hh_step = [&](const int j, auto tlo_c) {
            constexpr int TLO = decltype(tlo_c)::value;
            __builtin_amdgcn_s_setprio(2);    // the reflector's serial part issues first
            __syncthreads();                  // column j is in colb, its row-group norms in nrmp
            double2 x[NI];
#pragma unroll
            for (int z = 0; z < NI; ++z) {
                const int i = lam + z * L;
                x[z] = (i > j && i < s) ? colb[i] : cz();
            }
            const double2 alpha = colb[j + 1];
            // squared norm below the subdiagonal; rows past s are zero in the tile
            const double sig = tree_sum_d<P>(nrmp);
            const double tot = fma(alpha.x, alpha.x, fma(alpha.y, alpha.y, sig));
            // inputs are pre-scaled to entries of order one, so a column whose squared norm is
            // below 2^-660 is rounding noise of an already reduced (rank-deficient) part:
            // leave it (the bound also keeps 1 / (beta |alpha - beta|^2) below 2^990)
            const bool skip = tot < 0x1p-660 || (sig == 0.0 && alpha.y == 0.0);
            double2 tau = cz(), v[NI];
#pragma unroll
            for (int z = 0; z < NI; ++z) v[z] = cz();
            double bet = alpha.x;
            if (!skip) {
                // reflector P = I - tau v v^H with v unnormalised: v_{j+1} = d = alpha - beta,
                // v_r = x_r below it, tau = -1 / (beta conj(d)) = -d / (beta |d|^2); the same P
                // as v_{j+1} = 1, tau = (beta - alpha) / beta, for one reciprocal instead of three divisions
                const double nrm = sqrt_pos(tot);
                bet = alpha.x >= 0.0 ? -nrm : nrm;
                const double2 d = make_double2(alpha.x - bet, alpha.y);
                const double rb = -rcp_normal(bet * fma(d.x, d.x, d.y * d.y));
                tau = cscale(d, rb);
#pragma unroll
                for (int z = 0; z < NI; ++z) {
                    const int i = lam + z * L;
                    v[z] = i == j + 1 ? d : (i > j + 1 ? x[z] : cz());
                }
            }
#pragma unroll
            for (int z = 0; z < NI; ++z)
                if (lam + z * L < SM) vv[lam + z * L] = v[z];
            if (lam == 0) beta[j + 1] = skip ? alpha : make_double2(bet, 0.0);
            __syncthreads();
            double2 vr[R];
#pragma unroll
            for (int t = 0; t < R; ++t) vr[t] = (a + P * t < SM) ? vv[a + P * t] : cz();
            const int ulo = (j + 1) / Q;      // column slots left of ulo hold only columns <= j

            __builtin_amdgcn_s_setprio(0);
            // one pass: w partials (over own rows) and y partials (over own columns)
            double2 yp[R];
#pragma unroll
            for (int t = 0; t < R; ++t) yp[t] = cz();
#pragma unroll
            for (int u = 0; u < C; ++u)
                if (u >= ulo) {
                    const double2 vcu = (b + Q * u < SM) ? vv[b + Q * u] : cz();
                    double2 wp = cz();
#pragma unroll
                    for (int t = 0; t < R; ++t) {
                        if (t >= TLO) cfma_cj(wp, vr[t], h[t][u]);
                        cfma(yp[t], h[t][u], vcu);
                    }
                    wpart[b + Q * u + S::WA * a] = wp;
                }
#pragma unroll
            for (int t = 0; t < R; ++t) ypart[a + P * t + S::YB * b] = yp[t];
            __builtin_amdgcn_s_setprio(2);
            __syncthreads();
            // lane lam owns column and row lam (and lam + L): their w and y sums
            double2 w[NI], y[NI];
#pragma unroll
            for (int z = 0; z < NI; ++z) {
                const int i = lam + z * L;
                w[z] = (i > j && i < s) ? tree_sum<P, S::WA>(wpart + i) : cz();
                y[z] = i < s ? tree_sum<Q, S::YB>(ypart + i) : cz();
            }
            double2 wv = cmul(w[0], v[0]);
#pragma unroll
            for (int z = 1; z < NI; ++z) wv = cadd(wv, cmul(w[z], v[z]));
            const double2 gam = make_double2(group_sum<L>(wv.x), group_sum<L>(wv.y));
#pragma unroll
            for (int z = 0; z < NI; ++z) {
                const int i = lam + z * L;
                double2 y1 = y[z];
                cfms(y1, cmul(cconj(tau), gam), v[z]);
                if (i < SM) {
                    wb[i] = cmul(cconj(tau), w[z]);
                    yb[i] = cmul(tau, y1);
                }
            }
            __syncthreads();
            double2 yr[R];
#pragma unroll
            for (int t = 0; t < R; ++t) yr[t] = (a + P * t < SM) ? yb[a + P * t] : cz();
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int u = 0; u < C; ++u)
                if (u >= ulo) {
                    const double2 wu = (b + Q * u < SM) ? wb[b + Q * u] : cz();
                    const double2 vcu = (b + Q * u < SM) ? vv[b + Q * u] : cz();
#pragma unroll
                    for (int t = 0; t < R; ++t) {
                        if (t >= TLO) cfms(h[t][u], vr[t], wu);
                        cfms_cj(h[t][u], yr[t], vcu);
                    }
                }
            __builtin_amdgcn_s_setprio(2);
            // column j+1 -> colb and its norm below row j+2 -> nrmp for the next step
            // (its owners have just updated it)
            const int un = (j + 1) / Q, bn = (j + 1) % Q;
            if (b == bn && j + 3 < s) {
#pragma unroll
                for (int u = 0; u < C; ++u)
                    if (u == un) {
                        double part = 0.0;
#pragma unroll
                        for (int t = 0; t < R; ++t) {
                            if (a + P * t < SM) colb[a + P * t] = h[t][u];
                            if (a + P * t >= j + 3) part = fma(h[t][u].x, h[t][u].x, fma(h[t][u].y, h[t][u].y, part));
                        }
                        nrmp[a] = part;
                    }
            }
        };
        // One copy of the step per phase, phase PH running the steps with (j + 1) / P == PH
        // (row slots below PH hold rows <= j), where the copies do not cost more registers and
        // time than the skipped terms save: the tiles up to 4 x 4, and the 3 x 6 and 5 x 5
        // tiles without the loop moments (which leave them the registers).  Chosen by measurement.
        constexpr bool PHASED = R * C <= 16 || (!LOOPS && ((R == 3 && C == 6) || (P == 8 && Q == 8 && R == 5 && C == 5)));
        if constexpr (PHASED) {
            static_for<R>([&](auto ph) {
                constexpr int PH = decltype(ph)::value;
                const int jlo = PH == 0 ? 0 : PH * P - 1;
                const int jhi = PH == R - 1 ? s - 2 : min(s - 2, (PH + 1) * P - 1);
                for (int j = jlo; j < jhi; ++j) hh_step(j, std::integral_constant<int, PH>{});
            });
        } else {
            for (int j = 0; j + 2 < s; ++j) hh_step(j, std::integral_constant<int, 0>{});
        }
        __builtin_amdgcn_s_setprio(2);        // table, scaling walk: LDS latency chains
        // ---- the last subdiagonal entry (no reflector acts on it)
#pragma unroll
        for (int t = 0; t < R; ++t)
#pragma unroll
            for (int u = 0; u < C; ++u)
                if (a + P * t == s - 1 && b + Q * u == s - 2) beta[s - 1] = h[t][u];
        __syncthreads();                      // partial areas are free again
        // ---- upper triangle (incl. diagonal) -> packed table, column c holds rows 0..c
#pragma unroll
        for (int t = 0; t < R; ++t)
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const int r = a + P * t, c = b + Q * u;
                if (r <= c && c < s) red[c * (c + 1) / 2 + r] = h[t][u];
            }
        __syncthreads();
        for (int z = lam; z < S::SLACK; z += L) red[s * (s + 1) / 2 + z] = cz();   // slack after the table
        // g_{r,c+1} = h_{r,c} prod_{k=r+1}^{c} h_{k,k-1}: lane r walks its row (and row
        // r + L); the trip count is the same for every lane (lanes join at c = r), so
        // the loop unrolls and the reads of the next subdiagonal entries are issued early
        {
            double2 pi[NI];
#pragma unroll
            for (int z = 0; z < NI; ++z) pi[z] = cone();
#pragma unroll 4
            for (int c = 0; c < s; ++c) {
                const double2 bc = beta[c + 1 < s ? c + 1 : 0];
#pragma unroll
                for (int z = 0; z < NI; ++z) {
                    const int r = lam + z * L;
                    if (c >= r && r < s) {
                        const int idx = c * (c + 1) / 2 + r;
                        red[idx] = cmul(red[idx], pi[z]);
                        pi[z] = cmul(pi[z], bc);
                    }
                }
            }
        }
        __syncthreads();

        __builtin_amdgcn_s_setprio(0);
        // ---- characteristic polynomials
        if (CP == 0) {                        // each group: lane lam = degree d
            double2 cs = cz();
            switch (s) {
#define HAF_CP_CASE(SS) case SS: if (SS <= SM && SS + 8 > SM) \
                cs = charpoly_lanes<(SS <= SM ? SS : 2), 1, 0>(red, lam, 0, 0, nullptr, nullptr, 0); break;
                HAF_CP_CASES
#undef HAF_CP_CASE
                default: break;
            }
            write_coefs<NTS>(coef, cstride, valid, sub, s, N, lam, L, cs);
        } else if (CP == 1) {                 // whole wave per matrix, rows split over groups
#pragma unroll 1
            for (int gg = 0; gg < W; ++gg) {
                const int subg = (grp0 + gg) * span + q;
                const double2* gt = lds + gg * S::PER;
                double2 cs = cz();
                switch (s) {
#define HAF_CP_CASE(SS) case SS: if (SS <= SM && SS + 8 > SM) \
                    cs = charpoly_lanes<(SS <= SM ? SS : 2), W, 0>(gt, lam, g, 0, nullptr, nullptr, 0); break;
                    HAF_CP_CASES
#undef HAF_CP_CASE
                    default: break;
                }
                if (g == 0) write_coefs<NTS>(coef, cstride, subg < count, subg, s, N, lam, L, cs);
            }
        } else if (CP == 3) {                 // groups in pairs: each 32-lane half over one matrix's degrees
            const int half = tid >> 5, dd = tid & 31;
#pragma unroll 1
            for (int pr = 0; pr < W / 2; ++pr) {
                const int gg = 2 * pr + half;
                const int subg = (grp0 + gg) * span + q;
                const double2* gt = lds + gg * S::PER;
                double2 cs = cz();
                switch (s) {
#define HAF_CP_CASE(SS) case SS: if (SS <= SM && SS + 8 > SM) \
                    cs = charpoly_lanes<(SS <= SM ? SS : 2), 1, 0>(gt, dd, 0, 0, nullptr, nullptr, 0); break;
                    HAF_CP_CASES
#undef HAF_CP_CASE
                    default: break;
                }
                write_coefs<NTS>(coef, cstride, subg < count, subg, s, N, dd, 32, cs);
            }
        } else {                              // W == 1: degree passes d < 32, then d >= 32
            const int hh = lam / 32, dd = lam % 32;
            double2* bnd = beta;              // c_i[31] for every i (beta is no longer needed)
            double2 cs = cz();
            switch (s) {
#define HAF_CP_CASE(SS) case SS: if (SS <= SM && SS + 8 > SM) \
                cs = charpoly_lanes<(SS <= SM ? SS : 2), 2, 0>(red, dd, hh, 0, nullptr, bnd, 31); break;
                HAF_CP_CASES
#undef HAF_CP_CASE
                default: break;
            }
            if (hh == 0) write_coefs_range<NTS>(coef, cstride, valid, sub, s, N, dd, 0, 32, cs);
            if (s > 32) {
                __syncthreads();              // bnd is complete
                double2 cs2 = cz();
                switch (s) {
#define HAF_CP_CASE(SS) case SS: if (SS <= SM && SS + 8 > SM && SS > 32) \
                    cs2 = charpoly_lanes<(SS <= SM && SS > 32 ? SS : 34), 2, 32>(red, dd + 32, hh, 32, bnd, nullptr, 0); break;
                    HAF_CP_CASES
#undef HAF_CP_CASE
                    default: break;
                }
                if (hh == 0) write_coefs_range<NTS>(coef, cstride, valid, sub, s, N, dd + 32, 32, s, cs2);
            }
            if (hh == 0 && valid)
                for (int kk = s + 1 + dd; kk <= N; kk += 32) store_coef<NTS>(&coef[(int64_t)(kk - 1) * cstride + sub], cz());
        }
        __syncthreads();                      // LDS is reused by the next subset
    }
}


// Layouts and the subset sizes each one serves: (P, Q, R, C, CP) for s in (lo, hi].
// The table packs two or four matrices per wave where the tile fits, in steps of
// 4 rows from 8 up to 32 so that little of a tile is padding.  A layout can serve
// any s in (SM - 8, SM] (the polynomial stage is instantiated for those sizes),
// and two layouts with the same P, Q and CP give bitwise the same results for a
// subset (padded rows and columns only add exact zeros; every sum runs over the
// same P or Q partials in the same order).
#define HAF_REG_TABLE(X) X(4, 4, 2, 2, 0, 0, 8) X(4, 4, 3, 3, 0, 8, 12) X(4, 4, 4, 4, 0, 12, 16)       \
                          X(4, 4, 5, 5, 3, 16, 20) \
                          X(8, 4, 3, 6, 0, 20, 24) X(8, 4, 4, 7, 1, 24, 28) X(8, 4, 4, 8, 1, 28, 32)      \
                          X(8, 8, 5, 5, 2, 32, 40) X(8, 8, 6, 6, 2, 40, 48)

}  // namespace hafgpu
