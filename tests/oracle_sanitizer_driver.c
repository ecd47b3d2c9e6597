/* Driver for the oracle under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Test infrastructure: compiled together with oracle/haf_oracle.c by
 * tests/test_oracle_sanitizers.py and run on the CPU.  It reads one binary input
 * file (argv[1]):
 *     int32 n, then n*n complex doubles (re, im) of a symmetric matrix A;
 *     int32 g, then g*g int64 entries of an integer matrix G;
 *     int32 k, then k*k complex doubles of a square matrix W;
 * calls every exported oracle routine on them and prints one line per result
 * (doubles with 17 significant digits), for comparison with the ordinary build. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_formula_range(const double* A, int n, int loops, int prec, uint64_t lo, uint64_t hi, int nthreads,
                      double* out, double* absum);
int orc_formula_masks(const double* A, int n, int loops, int prec, const uint32_t* masks, int64_t count,
                      int nthreads, double* out);
int orc_term(const double* A, int n, int loops, int prec, uint32_t mask, double* out);
int orc_ryser(const double* W, int k, int prec, int nthreads, double* out);
int orc_brute(const double* A, int n, int loops, double* out);
int orc_brute_int(const int64_t* A, int n, int loops, uint64_t* out);
int orc_modp(const int64_t* A, int n, int loops, uint64_t p, int nthreads, uint64_t* out);
int orc_modp_term(const int64_t* A, int n, int loops, uint64_t p, uint32_t mask, uint64_t* out);

static void* read_block(FILE* f, size_t bytes) {
    void* p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static int read_dim(FILE* f) {
    int32_t d = 0;
    if (fread(&d, sizeof d, 1, f) != 1 || d < 0 || d > 64) {
        fprintf(stderr, "bad dimension\n");
        exit(2);
    }
    return d;
}

static void print4(const char* tag, int a, int b, const double* r) {
    printf("%s %d %d %.17g %.17g %.17g %.17g\n", tag, a, b, r[0], r[1], r[2], r[3]);
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    const int n = read_dim(f);
    double* A = (double*)read_block(f, sizeof(double) * 2 * (size_t)n * n);
    const int g = read_dim(f);
    int64_t* G = (int64_t*)read_block(f, sizeof(int64_t) * (size_t)g * g);
    const int k = read_dim(f);
    double* W = (double*)read_block(f, sizeof(double) * 2 * (size_t)k * k);
    fclose(f);

    double r[4], ab = 0.0;
    const int N = n / 2;
    for (int loops = 0; loops <= 1; ++loops) {
        if (orc_brute(A, n, loops, r)) return 3;
        print4("brute", loops, 0, r);
        for (int prec = 0; prec <= 3; ++prec) {
            if (orc_formula_range(A, n, loops, prec, 1, (uint64_t)1 << N, 2, r, &ab)) return 3;
            print4("formula", loops, prec, r);
            printf("absum %d %d %.17g\n", loops, prec, ab);
            const uint32_t mask = ((uint32_t)1 << N) - 1u - 2u;
            if (orc_term(A, n, loops, prec, mask, r)) return 3;
            print4("term", loops, prec, r);
        }
        uint32_t masks[5] = { 1u, 3u, 6u, ((uint32_t)1 << N) - 1u, 5u };
        if (orc_formula_masks(A, n, loops, 1, masks, 5, 2, r)) return 3;
        print4("masks", loops, 1, r);
        uint64_t bi[2];
        if (orc_brute_int(G, g, loops, bi)) return 3;
        printf("brute_int %d %llu %llu\n", loops, (unsigned long long)bi[0], (unsigned long long)bi[1]);
        uint64_t v = 0;
        if (orc_modp(G, g, loops, 2147483647ull, 2, &v)) return 3;
        printf("modp %d %llu\n", loops, (unsigned long long)v);
        if (orc_modp_term(G, g, loops, 2147483629ull, 5u, &v)) return 3;
        printf("modp_term %d %llu\n", loops, (unsigned long long)v);
    }
    for (int prec = 0; prec <= 3; ++prec) {
        if (orc_ryser(W, k, prec, 2, r)) return 3;
        print4("ryser", prec, 0, r);
    }
    free(A);
    free(G);
    free(W);
    return 0;
}
