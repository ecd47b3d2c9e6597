/*
 * hafgpu -- hafnians and loop hafnians of complex symmetric matrices on AMD
 * Instinct MI355X (gfx950), behind a plain C ABI.
 *
 * Method: the inclusion-exclusion formula over the 2^(n/2) subsets Z of the
 * vertex pairs (2i, 2i+1) (Sec. 3.2, Eq. Pset), each term
 *     f(Z) = [lambda^(n/2)] exp( sum_k ( tr(B^k) / (2k) [+ l_k / 2] ) lambda^k )
 * with B the submatrix of X*A on the rows/columns of Z (Eq. matA, Eq. poly,
 * Eq. haffinal; X swaps the two vertices of each pair) and, for the loop
 * hafnian, the loop moments l_k = d^T B^(k-1) X d of the diagonal d (the loop
 * formula of Sec. 3.3, read as the walk count of Sec. 3.1).  The power traces
 * come from a Hessenberg reduction and the characteristic polynomial
 * (App. B).  Every step runs in complex double on the GPU; the signed outer
 * sum is accumulated in double-double.
 *
 * Data layout: a matrix is row-major interleaved complex128 (haf_cplx,
 * byte-compatible with numpy / torch complex128), element (i, j) at
 * A[i * lda + j], lda >= n.
 *
 * Errors: every entry point returns an int status (HAF_OK = 0 or a HAF_E_*
 * code) and never throws; haf_last_error() gives a thread-local message.
 *
 * Streams are passed as void* and are hipStream_t values (NULL = the null
 * stream).  Entry points named *_dev take device pointers, enqueue work on the
 * stream and return without waiting; the caller keeps inputs and outputs alive
 * until the stream passes the call.  Host entry points (no _dev suffix) copy in,
 * run and copy out synchronously, and keep nothing after returning.
 */
#ifndef HAFGPU_H
#define HAFGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } haf_cplx;
/* a complex value as unevaluated sums re_hi + re_lo, im_hi + im_lo (double-double) */
typedef struct { double re_hi, re_lo, im_hi, im_lo; } haf_cplx2;

enum {
    HAF_OK = 0,
    HAF_E_INVALID_ARG = 1,   /* null pointer, n < 0, lda < n, unknown kind, count < 0 */
    HAF_E_TOO_LARGE = 2,     /* n > HAF_MAX_N (after padding an odd n for lhaf)      */
    HAF_E_NOT_SYMMETRIC = 3, /* A[i][j] != A[j][i] exactly (the method assumes A = A^T, Sec. 2) */
    HAF_E_NONFINITE = 4,     /* NaN or Inf entry                                      */
    HAF_E_DEVICE = 5,        /* a HIP call failed                                     */
    HAF_E_NOMEM = 6,         /* device or host allocation failed                      */
    HAF_E_BUSY = 7,          /* serving: no free request slot and the queue is full  */
    HAF_E_STATE = 8          /* serving: unknown ticket / server stopped              */
};

#define HAF_MAX_N 64         /* subset masks are 32-bit and a subset matrix fits one 64-lane wave */
#define HAF_KIND_HAF 0
#define HAF_KIND_LHAF 1

/* Thread-local text of the last error on this thread ("" if none). */
const char* haf_last_error(void);

/* Library version string. */
const char* haf_version(void);

/* Select and initialise a HIP device for this thread's subsequent calls
 * (optional: the current device is initialised lazily).  Also loads the batched
 * configuration cached for this device, if HAF_AUTOTUNE_CACHE names a file that
 * has one (haf_batched_load_cache).
 *
 * Environment (read by the library):
 *   HAF_AUTOTUNE_CACHE  file of tuned batched configurations, one per device;
 *   HAF_ARENA_BYTES     default server arena (integer, optional K/M/G suffix);
 *   HAF_KERNEL_PATH     initial kernel path (0, 1 or 2; haf_set_kernel_path);
 *   HAF_DEBUG           non-zero: every error is also printed to stderr. */
int haf_init(int device);

/* One-line description of the device and kernel configuration into buf. */
int haf_device_info(char* buf, int buflen);

/*
 * haf(A) (Sec. 2, Eq. hafA), host pointers, synchronous.  The diagonal of A is
 * ignored.  n = 0 gives 1, odd n gives 0.  A must be exactly symmetric and
 * finite.  n <= 64.
 */
int haf_c128(const haf_cplx* A, int n, int lda, haf_cplx* out);

/*
 * lhaf(A) (the loop hafnian of Sec. 2; diagonal entries are loop weights),
 * host pointers, synchronous.  Odd n is computed as lhaf(A (+) [1]) (an
 * isolated vertex whose loop has weight 1).  n <= 63 for odd n, 64 for even.
 */
int lhaf_c128(const haf_cplx* A, int n, int lda, haf_cplx* out);

/* Either kind (HAF_KIND_HAF / HAF_KIND_LHAF), result as double-double. */
int haf_c128x2_host(const haf_cplx* A, int n, int lda, int kind, haf_cplx2* out);

/*
 * perm(W) of an n x n complex matrix through the bipartite identity
 * (Sec. 1.1): perm(W) = haf(B) for the 2n x 2n matrix B = [[0, W], [W^T, 0]]
 * of the complete bipartite graph with edge weights W.  Host pointers,
 * synchronous; W is read row-major with leading dimension ldw >= n and must be
 * finite.  n = 0 gives 1; n <= 32 (HAF_E_TOO_LARGE above).  The result is the
 * hafnian path's result for B, bit for bit.
 */
int perm_c128(const haf_cplx* W, int n, int ldw, haf_cplx* out);
/* Device variant: dW is a device matrix (not inspected), d_out a device
 * haf_cplx; B is built on `stream` in the library's workspace for that stream. */
int perm_c128_dev(const haf_cplx* dW, int n, int ldw, haf_cplx* d_out, void* stream);

/*
 * Device variants: dA is a device matrix, d_out a device haf_cplx (or
 * haf_cplx2 for the x2 form).  Only n, lda and the pointers are checked; the
 * matrix contents are not inspected (they are on the device), so the caller
 * guarantees symmetry.  Scratch memory comes from a library-owned pool kept per
 * (device, stream); it is allocated or grown on first use and kept until
 * haf_release_workspaces().
 */
int haf_c128_dev(const haf_cplx* dA, int n, int lda, haf_cplx* d_out, void* stream);
int lhaf_c128_dev(const haf_cplx* dA, int n, int lda, haf_cplx* d_out, void* stream);
int haf_c128x2_dev(const haf_cplx* dA, int n, int lda, int kind, haf_cplx2* d_out, void* stream);

/*
 * Allocation-free variant of haf_c128x2_dev, for callers that cannot allocate
 * device memory (code under stream or graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, same launch sequence and
 * bitwise the same result as haf_c128x2_dev; every work buffer (exponent,
 * padded odd-n matrix, partial slots, coefficients) comes from one fixed
 * 80 MiB array in device memory that the library holds on each device it runs
 * on until the process ends, so the call performs no allocation of any kind.
 * Limit: n <= 56 (after padding an odd n for lhaf); larger n return
 * HAF_E_TOO_LARGE (the partial slots of n = 58 alone exceed the array).  Every
 * call on one device uses the same array, so calls that overlap on a device
 * (on different streams, or from different threads without ordering) race
 * and give wrong results; calls ordered on one stream are safe.  The array
 * keeps the last call's contents; nothing in it needs clearing between calls.
 */
int haf_c128x2_dev_noalloc(const haf_cplx* dA, int n, int lda, int kind, haf_cplx2* d_out, void* stream);

/*
 * The unsigned terms f(Z) (Sec. 3.3, Eq. haffinal without the outer sum) for
 * the subsets given as bit masks over the n/2 pairs (bit i = pair (2i, 2i+1)).
 * d_masks: device uint32[count]; d_terms: device haf_cplx[count].  Exposes the
 * per-subset stage for sampled checks at sizes where the full sum is out of
 * reach of a CPU reference.  n even, 2 <= n <= 64, masks nonzero and < 2^(n/2).
 */
int haf_terms_dev(const haf_cplx* dA, int n, int lda, int kind, const uint32_t* d_masks, int count,
                  haf_cplx* d_terms, void* stream);

/*
 * Per-term double-double precision mode (opt-in): the same route as the
 * device and host entry points (Householder Hessenberg form, characteristic
 * polynomial, Newton's identities, exponential series), but every step of each
 * term f(Z) in complex double-double (about 106 significant bits) instead of
 * complex double.  The paper's precision ablation (Sec. 4.2) shows that the
 * precision of the terms, not the outer summation, sets the error of the
 * alternating sum; with double-double terms the error bound drops from
 * ~eps64 * kappa to ~eps_dd * kappa (kappa = sum_Z |f(Z)| / |haf|).  About an
 * order of magnitude more work per term.  Arguments, layout, edge cases and
 * errors as haf_c128x2_dev / haf_c128x2_host; the result is double-double.
 */
int haf_dd_c128x2_dev(const haf_cplx* dA, int n, int lda, int kind, haf_cplx2* d_out, void* stream);
int haf_dd_c128x2_host(const haf_cplx* A, int n, int lda, int kind, haf_cplx2* out);

/*
 * Exact hafnian / loop hafnian of an integer matrix (row-major int64, leading
 * dimension lda >= n, exactly symmetric off the diagonal; haf ignores the
 * diagonal).  Each term f(Z) of the subset sum counts tangles and is an
 * integer (Sec. 3.2, Eq. Pset), and the route from B = X A_Z to f(Z) needs
 * only field operations (App. B), so the library runs the whole sum on the GPU
 * modulo primes p < 2^25 (the largest ones below 2^25) and reconstructs the
 * integer by Chinese remaindering: enough primes for a product above twice a
 * bound on |haf| ((n-1)!! max|a_ij|^(n/2); T(n) max(sqrt(max|a_ij|),
 * max|a_ii|)^n for lhaf), plus one more prime that must agree.  Host pointers,
 * synchronous.  The value is returned as sign (-1, 0, 1) and magnitude, eight
 * 32-bit limbs, least significant first.  n = 0 gives 1, odd n gives 0 for
 * haf and lhaf(A (+) [1]) for lhaf.  Errors: HAF_E_INVALID_ARG,
 * HAF_E_NOT_SYMMETRIC, HAF_E_TOO_LARGE (n > 64, or a bound that needs more than
 * ten primes, e.g. n > 56 for dense 0/1 graphs), HAF_E_DEVICE (also if the
 * check prime disagrees), HAF_E_NOMEM.
 */
int haf_exact_i64(const int64_t* A, int n, int lda, int kind, uint32_t* magnitude, int* sign);
/* The same sum modulo each of the given primes (1..10 of them, each a prime
 * with n + 1 < p < 2^25; HAF_E_INVALID_ARG otherwise): residues[i] in [0, p_i). */
int haf_modp_c(const int64_t* A, int n, int lda, int kind, const uint32_t* primes, int nprimes, uint32_t* residues);

/*
 * Hafnian of a low-rank matrix from its factor (App. C): G is n x r (row-major,
 * leading dimension ldg >= r, complex, host memory), and the result is the
 * hafnian of any matrix whose entries above the diagonal are those of G G^T
 * (the hafnian ignores the diagonal).  With q(x) = prod_i (sum_j g_ij x_j) =
 * sum_p lambda_p x^p, haf = sum over even exponent vectors e of
 * lambda_e prod_j (e_j - 1)!!; the GPU expands q one factor at a time over the
 * C(n + r - 1, r - 1) monomials of each degree, so the cost is polynomial in
 * n for a fixed rank instead of 2^(n/2).  Synchronous; result as double-double;
 * *cond (if not null) receives sum_e |lambda_e| prod (e_j - 1)!! / |haf|, the
 * cancellation of the final sum.  n = 0 gives 1, odd n gives 0.  Errors:
 * HAF_E_INVALID_ARG (null pointer, n < 0, r < 1, ldg < r), HAF_E_TOO_LARGE
 * (n > 64, r > 8, or more than 2^28 monomials of degree n), HAF_E_NONFINITE,
 * HAF_E_NOMEM, HAF_E_DEVICE.
 */
int haf_lowrank_c128(const haf_cplx* G, int n, int r, int ldg, haf_cplx2* out, double* cond);

/*
 * Batched: count independent hafnians / loop hafnians of uneven sizes (the
 * per-matrix sums of Sec. 3.2, Eq. Pset; the paper names batched small-matrix
 * GPU work as the way forward in its conclusions).  Matrix t is stored densely
 * (lda = n_t) at element offset h_offsets[t] of dA_packed (device memory).
 * h_offsets, h_n and h_kind (HAF_KIND_*) are host arrays (the plan is built on
 * the host from the sizes alone); d_out is a device haf_cplx[count] (haf_cplx2
 * for the x2 form).  Asynchronous like the *_dev calls: the work is ordered
 * after everything already on `stream`, and `stream` does not pass the call
 * until every result is written.
 *
 * With haf_batched_config.grouped = 1 (default) every matrix with n <= 32
 * (after padding odd-n loop hafnians) runs in launches shared by the whole
 * batch, on `stream`: one prologue (constant results, padding, input scaling),
 * then per register layout and kind one coefficient launch over the subset
 * size classes of every matrix that layout serves and one series launch over
 * the same chunks, then one reduction launch.  Matrices above 32 rows (and,
 * with grouped = 0, every matrix) run the single-matrix path spread, largest
 * model cost first, over haf_batched_config.streams library streams.  Either
 * way each matrix keeps the single-matrix path's per-subset arithmetic,
 * partial slots and reduction order, so every result is bitwise the
 * single-matrix path's result for that matrix, whatever else is in the batch
 * and whatever the configuration.
 * Errors: HAF_E_INVALID_ARG (null pointer, count < 0, n_t < 0, unknown kind),
 * HAF_E_TOO_LARGE (n_t > HAF_MAX_N), HAF_E_NOMEM, HAF_E_DEVICE.  Matrices are
 * not checked for symmetry (they live in device memory).
 */
int haf_batched_c128(const haf_cplx* dA_packed, const int64_t* h_offsets, const int32_t* h_n,
                     const uint8_t* h_kind, int count, haf_cplx* d_out, void* stream);
int haf_batched_c128x2(const haf_cplx* dA_packed, const int64_t* h_offsets, const int32_t* h_n,
                       const uint8_t* h_kind, int count, haf_cplx2* d_out, void* stream);

/* Tunable parameters of the batched path (process-wide).  No setting changes a result. */
typedef struct {
    int table;          /* layouts of the shared coefficient launches: 0 (default) the
                           single-matrix table (nine layouts), 1 four coarse layouts (fewer
                           launches, more padded rows)                                   */
    int span;           /* subsets each lane group takes in a shared coefficient launch,
                           1..64 (default 4): fewer unrankings against a coarser split    */
    int streams;        /* streams for the matrices above 32 rows, 1..4 (default 4)      */
    int grouped;        /* 1 (default): shared launches for n <= 32; 0: single-matrix
                           launches for every matrix                                     */
    int coef_budget_mb; /* device memory for the coefficients of one shared launch pair,
                           MiB, 64..262144 (default 8192); a larger stage is cut into
                           several launch pairs                                          */
} haf_batched_config;

int haf_batched_get_config(haf_batched_config* cfg);
/* HAF_E_INVALID_ARG for values out of range. */
int haf_batched_set_config(const haf_batched_config* cfg);
/* Autotuner: runs the given batch (same arguments as haf_batched_c128; d_out
 * receives the results) under a coordinate search (span 1..16 with the full
 * layout table, then the other table, then 1, 2, 4 streams, then grouped = 0),
 * times each run with HIP events on `stream`, makes the fastest the current
 * configuration and returns it in *best and its time in *best_ms.  Synchronous.
 * If HAF_AUTOTUNE_CACHE names a file, the result is also stored there as this
 * device's entry (one text line "<arch>:<CUs> table span streams grouped
 * coef_budget_mb", replacing an older one); HAF_E_STATE if the file cannot be
 * written (the configuration is applied all the same). */
int haf_batched_tune(const haf_cplx* dA_packed, const int64_t* h_offsets, const int32_t* h_n,
                     const uint8_t* h_kind, int count, haf_cplx* d_out, void* stream, haf_batched_config* best,
                     double* best_ms);
/* Make the current device's entry of the HAF_AUTOTUNE_CACHE file the current
 * batched configuration.  HAF_E_STATE if the variable is unset or the file has
 * no entry for this device, HAF_E_INVALID_ARG for a malformed line or values
 * out of range, HAF_E_DEVICE without a device. */
int haf_batched_load_cache(void);
/* Host-only view of the shared launches under the current configuration (no
 * device needed).  launches receives 8 int64 per launch, in launch order:
 * (what: 0 coefficients / 1 series, layout, loops, blocks, first chunk, chunks,
 * coefficient storage in complex values, largest s of the layout); chunks
 * receives 8 int64 per chunk: (matrix index, m, subsets, first block, coefficient
 * offset, first partial slot, N, first rank).  Matrices that do not take the
 * shared launches appear in neither.  At most max_launches / max_chunks
 * entries are written; *n_launches and *n_chunks receive the full counts. */
int haf_batched_plan(const int32_t* h_n, const uint8_t* h_kind, int count, int64_t* launches, int max_launches,
                     int* n_launches, int64_t* chunks, int max_chunks, int* n_chunks);

/* Free every cached workspace of every device (waits for the device first). */
int haf_release_workspaces(void);

/* Kernel path selection (for testing and tuning): 0 = automatic (for n <= 32
 * all size classes of a matrix go out in one coefficient launch per layout and
 * one series launch), 1 = LDS kernel only, 2 = register-tiled kernels, one
 * launch pair per size class (bitwise the results of 0).  All reach the same
 * characteristic polynomial (any similarity does, App. B); 1 differs from 0
 * and 2 in rounding.  Process-wide. */
int haf_set_kernel_path(int path);

/* ------------------------------------------------------------------------ */
/* Kernel timing.  While enabled, every coefficient launch (the per-subset
 * Hessenberg / characteristic-polynomial stage) and every series launch is
 * bracketed by HIP events recorded on the launch's own stream.                */
typedef struct {
    int64_t coef_launches;      /* coefficient kernel launches                         */
    double coef_ms;             /* summed event time of those launches                 */
    double coef_model_flops;    /* model flops of the subsets they processed:
                                   (44/3) s^3 per subset, + 8 (N-1) s^2 for loop hafnians */
    int64_t coef_subsets;       /* subsets they processed                              */
    int64_t series_launches;
    double series_ms;
    int64_t batched_launches;   /* coefficient launches shared by the matrices of a batch */
    double batched_ms;
    double batched_model_flops; /* same flop model over the subsets they processed      */
} haf_profile;

/* Start (on != 0) or stop recording; starting clears earlier records. */
int haf_profile_enable(int on);
/* Wait for the recorded launches and sum their times into *out. */
int haf_profile_read(haf_profile* out);

/* ------------------------------------------------------------------------ */
/* Serving: a continuous-batching request server.
 *
 * submit() validates the matrix (as the host entry points do), copies it and
 * queues it; it never waits for the device.  The server's scheduler thread
 * admits queued requests in arrival order whenever a request slot is free and
 * the device arena holds the request's whole device state: its matrix, the
 * padded copy of an odd-n loop hafnian, the exponent of its input scaling and
 * its partial slots (32 bytes per 256 subsets).  The other device memory of a
 * server (the tick coefficient buffer of tick_coef_bytes and small tick tables)
 * is allocated once at start.  Work runs in ticks on one stream: a tick takes
 * runs of subsets of one size class (cut at 256-subset boundaries) from every
 * admitted request, round-robin in admission order, up to tick_flops model
 * flops (44/3 s^3 per subset of s rows, + 8 (N-1) s^2 for loop hafnians) and
 * tick_coef_bytes of coefficients, and launches them together: one prologue for
 * the requests that start, one coefficient launch per register layout and kind,
 * one series launch per kind, one reduction for the requests that finish.  Two
 * ticks are enqueued ahead, so requests that arrive while a tick runs join the
 * next one, small requests finish within a tick or two of admission, and large
 * ones proceed a share of the budget per tick.  A result is bitwise the
 * single-matrix path's result for that matrix, whatever else the server runs.
 * Results are collected with poll().  With continuous = 0 the server runs one
 * request at a time through the single-matrix path (the plain server; its
 * single-matrix workspaces come on top of the arena).                        */
typedef struct haf_server haf_server;

typedef struct {
    int device;                 /* HIP device ordinal                                  */
    int64_t arena_bytes;        /* device bytes for the state of admitted requests     */
    int max_active;             /* request slots                                       */
    int max_queue;              /* host queue length before submit returns HAF_E_BUSY   */
    double tick_flops;          /* model flops of the work one tick launches (> 0)     */
    int64_t tick_coef_bytes;    /* coefficient memory of one tick (>= 512 KiB)          */
    int continuous;             /* 1: ticks over every admitted request (continuous
                                   batching); 0: one request at a time through the
                                   single-matrix path, in arrival order (plain)         */
} haf_server_config;

typedef struct {
    uint64_t ticket;
    int status;                 /* HAF_OK, HAF_E_DEVICE (a launch of its tick failed),
                                   or HAF_E_STATE if the server stopped before
                                   admitting the request                                */
    int n, kind;
    haf_cplx value;
    double t_submit, t_admit, t_done;   /* seconds on the host steady clock (haf_now) */
} haf_result;

/* Fill *cfg with defaults (1 GiB arena, 256 slots, 2e10 flops and 256 MiB of
 * coefficients per tick, continuous). */
void haf_server_default_config(haf_server_config* cfg);
/* Start a server: allocates the arena and starts its scheduler thread.  NULL
 * on failure (haf_last_error() says why). */
haf_server* haf_server_create(const haf_server_config* cfg);
/* Copy the host matrix A and queue it; non-blocking.  *ticket identifies it.
 * Errors as for haf_c128, plus HAF_E_BUSY (queue full), HAF_E_NOMEM (the
 * request alone is larger than the arena), HAF_E_STATE (server stopping). */
int haf_server_submit(haf_server* s, const haf_cplx* A, int n, int lda, int kind, uint64_t* ticket);
/* Move up to max finished results into out; *n_out tells how many. */
int haf_server_poll(haf_server* s, haf_result* out, int max, int* n_out);
/* Block until every submitted request has finished. */
int haf_server_drain(haf_server* s);
/* Stop the scheduler and free its device memory (pending requests fail). */
void haf_server_destroy(haf_server* s);
/* Failure handling.  When a tick (or, in the plain server, a request's launch)
 * reports a HIP error, the scheduler waits for everything enqueued on its
 * stream, fails every admitted request with HAF_E_DEVICE, replaces the stream
 * with a new one and goes on admitting the queued requests.  This test hook
 * makes the next `count` completed ticks (plain server: requests) take that
 * path although their launches succeeded, so the recovery can be exercised
 * from the host without a device fault.  Returns HAF_E_INVALID_ARG for a null
 * server or a negative count. */
int haf_server_debug_fail_ticks(haf_server* s, int count);
/* Seconds on the steady clock used for the t_* fields. */
double haf_now(void);

#ifdef __cplusplus
}
#endif

#endif /* HAFGPU_H */
