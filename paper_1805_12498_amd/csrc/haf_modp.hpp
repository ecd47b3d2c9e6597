// The subset sum over prime fields: per-prime constants and launch wrappers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hafgpu {

constexpr int kModpMaxN = 32;               // n / 2 limit (n <= 64)
constexpr uint32_t kModpPrimeLimit = 1u << 25;

// Constants of one prime field F_p: p, 1/p (rounded) and the inverses of
// 0 .. 2 kModpMaxN (inv[0] unused) as integer-valued doubles.
struct ModpPrime {
    double p, pinv;
    double inv[2 * kModpMaxN + 2];
};

// Coefficients of det(I - lambda B) mod p (a_1..a_N at coef[(k-1) cstride + i]) and,
// for loops, l_1..l_N at coef[(N + k - 1) cstride + i], for subsets i = 0..count-1
// (ranks rank0.. of size class m), for every prime (blockIdx.y; prime i's area at
// coef + i * prime_stride; its matrix, reduced mod p, at Ap + i * n * n).
hipError_t launch_modp_coef(int s, bool loops, int grid, int nprimes, hipStream_t st, const double* Ap, int n, int N,
                            int m, uint64_t rank0, int count, const ModpPrime* primes, double* coef, int64_t cstride,
                            int64_t prime_stride);
// Series and signed block sums mod p: partial slot slot0 + b of each prime.
hipError_t launch_modp_series(bool loops, int count, int N, bool negative, int nprimes, hipStream_t st,
                              const double* coef, int64_t cstride, int64_t prime_stride, const ModpPrime* primes,
                              double* partials, int64_t slot0, int64_t slot_stride);
// residues[i] = sum of prime i's nslots partials mod p_i.
hipError_t launch_modp_reduce(int nprimes, hipStream_t st, const double* partials, int64_t nslots,
                              int64_t slot_stride, const ModpPrime* primes, double* residues);

}  // namespace hafgpu
