/*
 * pm.h -- C ABI of libpm: products of univariate polynomial matrices over
 * Z/pZ on one AMD Instinct MI355X (gfx950), by evaluation/interpolation.
 *
 * Operation (Hyun, Neiger, Schost, ISSAC 2019, Section 2, "Polynomial matrix
 * multiplication"): given A (m x n) and B (n x k) whose entries are
 * polynomials of degree < d over F_p (the set K[x]_d of Section 2,
 * "Polynomial multiplication"), compute C = A B (m x k, degree < 2d-1):
 *
 *   C[c][i][j] = sum_{l<n} sum_{a+b=c} A[a][i][l] * B[b][l][j]  (mod p),
 *   0 <= c <= 2d-2.
 *
 * Method (same section): evaluate A and B at the L-th roots of unity of a
 * prime q (L = 2^ceil(log2(2d-1))), multiply the m x n and n x k matrices
 * of values point by point, interpolate back (the number-theoretic
 * transform; Section 2, "Polynomial multiplication", FFT paragraph).
 *   * Direct mode: p itself is prime, p < 2^31 and 2^log2(L) divides p-1.
 *   * CRT mode, for any other modulus p >= 2 (the 3-primes idea of Section 2,
 *     "Polynomial multiplication" and "Polynomial matrix multiplication"):
 *     lift inputs to integers in [0, p), compute the integer product modulo
 *     r word-size NTT primes q_1..q_r with prod q_i > n*d*(p-1)^2, rebuild
 *     it by the Chinese remainder theorem (Garner) and reduce mod p.
 * Both modes return the exact product: no rounding, no tolerance.
 *
 * Layout (all operands, device memory, coefficient-major: the "polynomial
 * with matrix coefficients" representation that Section 3 describes after
 * the PM-IntBasis algorithm): a polynomial matrix with
 * R x S entries and D coefficients is D consecutive R x S row-major
 * matrices; element (c, i, j) sits at offset (c*R + i)*S + j.  A holds d*m*n
 * residues, B holds d*n*k, C receives (2d-1)*m*k.  Inputs must be canonical
 * residues in [0, p); other values give an unspecified (memory-safe) result;
 * pm_check_residues tests this on request.  Outputs are canonical.
 *
 * Ownership and streams: the caller owns A, B, C, the workspace and the
 * stream (a hipStream_t passed as void*, NULL for the default stream).
 * Every pm_mul* call only enqueues work on that stream and returns; results
 * are valid once the stream has completed.  Buffers must stay alive until
 * then.  The library allocates no device memory: its tables (roots of unity
 * per prime and length, Vandermonde matrices) live in regions of device
 * memory the caller registers with pm_tables_attach, are filled by a kernel
 * on the stream of the first call that needs them (no host copy, so a first
 * call may run inside a stream capture) and are reused by later calls on any
 * stream.  Calls from several host threads are safe; two calls that share a
 * workspace must be ordered on one stream.
 *
 * Errors: every argument check runs before anything is enqueued; a failed
 * check returns a negative pm_status and writes nothing.  A device fault is
 * reported as PM_EDEVICE by pm_sync or by a later call.  No C++ exception
 * crosses this interface (a failed host allocation is PM_ENOMEM) and the
 * library never aborts the process.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pm_status {
  PM_OK = 0,
  PM_EINVAL = -1,        /* bad argument: size < 1, NULL pointer, p < 2, overlap */
  PM_ERANGE = -2,        /* modulus or size outside what this API supports       */
  PM_ENOMEM = -3,        /* a host allocation of the library failed              */
  PM_EWORKSPACE = -4,    /* workspace NULL, misaligned or too small              */
  PM_EDEVICE = -5,       /* a HIP call failed                                    */
  PM_EUNSUPPORTED = -6,  /* no prime set covers the requested length/bound       */
  PM_EBUSY = -7,         /* reserved for admission control (serving layer)       */
  PM_ETABLES = -8,       /* no table region attached, or the regions are full    */
  PM_ESCRATCH = -9       /* pm_mul_noalloc: workspace beyond its static scratch  */
} pm_status;

/* Human-readable name of a status code (static string, never NULL). */
const char* pm_status_str(int status);

/* ABI version of this header; bumped on incompatible change. */
#define PM_ABI_VERSION 8
int pm_abi_version(void);

/* Plan of one product, computed on the host without touching the device.
 * mode: 0 = direct NTT mod p, 1 = CRT over num_primes NTT primes, 2 =
 * evaluation at 0 .. 2d-2 by Vandermonde products (pm_plan only: a CRT-mode
 * uint32 product that pm_mul_u32 sends through pm_mul_vdm_u32; primes and
 * log2_len then describe the CRT plan it replaces).
 * pointwise: 0 = VALU Barrett kernel, 1 = int8-MFMA limb kernel. */
typedef struct pm_plan_info {
  int32_t mode;
  int32_t log2_len;          /* L = 2^log2_len evaluation points            */
  int32_t num_primes;        /* 1 in direct mode                            */
  int32_t pointwise;
  uint32_t primes[8];        /* q_1..q_r (primes[0] = p in direct mode)     */
  uint64_t workspace_bytes;  /* what pm_mul_* needs for this product        */
  int32_t wrap_log2_len;     /* j > 0: pm_mul_* computes the product as
                                A B mod (x^(2^j) - 1) on 2^j points plus its
                                top coefficients from a short product (large
                                products with 2d - 1 a little above 2^j);
                                0: on 2^log2_len points                     */
  int32_t tune_entry;        /* index of the tuning-table entry whose launch
                                shapes the product uses; -1: the defaults   */
  int32_t num_points;        /* points the product is evaluated at: L, or
                                3L/4 when 2d - 1 <= 3L/4 (the roots of
                                (x^(L/2) - 1)(x^(L/4) - w^(L/4)), enough for
                                a product of fewer than 3L/4 coefficients) */
} pm_plan_info;

/* Tuning table (Section 2, "Polynomial matrix multiplication": thresholds
 * between variants are found experimentally, separately for small and large
 * primes).  Launch shapes per (prime class, log2 L, shape bucket): column-pass
 * stages, stages per block pass, block-step threads and tile, column item
 * widths, register or LDS block tile, MFMA or VALU pointwise, pipelined
 * pointwise slots; and global choices: batch tiles and thresholds (which
 * products of a batched call run on the single-product kernels), the
 * wrapped-length and three-quarter-length rules, whether CRT-mode products
 * fold the reconstruction into the last inverse pass and read their input
 * once for all primes, lazy butterfly ranges for small moduli, and how far
 * small single products spread over workgroups.  No choice changes a
 * result.  The table is JSON (format "pm-tune-1", written by
 * the tuning driver paper_1905_04356_amd/tune.py); it is read on first use
 * from $PM_TUNE_TABLE if set (empty: none), else from tune_table.json beside
 * libpm.so; a missing or invalid file leaves the defaults (PM_TUNE_*
 * environment variables, else built in).
 * pm_tune_load installs the table in `json` (NULL: read the default file
 * again; "": no table).  PM_EINVAL if the text is not a valid table (the
 * current one stays).  Calls in flight keep the shapes they were planned
 * with; cached batch graphs are rebuilt.  Host only.
 * pm_tune_info: number of entries, and where the table came from (0: none,
 * defaults; 1: the file; 2: pm_tune_load; -1: the file was invalid). */
pm_status pm_tune_load(const char* json);
pm_status pm_tune_info(int32_t* entries, int32_t* source);

/* Plan the product of an (m x n) by (n x k) matrix of degree < d mod p with
 * elem_bytes-byte residues (4 or 8).  Host only.  Returns PM_EINVAL on sizes
 * < 1, PM_ERANGE if p does not fit elem_bytes (p < 2^32 for 4, p < 2^62 for
 * 8) or if a size product overflows, PM_EUNSUPPORTED if L = 2^ceil(log2(2d-1))
 * exceeds 2^15 (transforms are held in on-chip memory) or no prime set
 * covers the CRT bound. */
pm_status pm_plan(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                  int32_t elem_bytes, pm_plan_info* out);

/* Device tables.  pm_tables_attach registers `bytes` of device memory at
 * dev_ptr (256-byte aligned, owned by the caller, on the current device) as
 * a region from which the library carves its tables; it must stay allocated
 * and untouched by the caller until the process ends or pm_tables_reset.
 * Several regions may be attached; a call whose missing tables do not fit
 * the free space of the attached regions returns PM_ETABLES before
 * enqueueing anything (attach another region and call again).  PM_EINVAL on
 * a NULL or misaligned pointer, fewer than 256 bytes, or overlap with an
 * attached region.
 * pm_tables_bytes: an upper bound of the table bytes a pm_mul_* call of this
 * product carves the first time (every (prime, length) pair it may use,
 * including the wrapped form and the Vandermonde route); a table shared by
 * several products is carved once.
 * pm_tables_reset: forget every table and region of the current device (for
 * tests and for releasing the regions); no work that reads them may be in
 * flight or captured in a graph that is still launched.
 * pm_tables_info: bytes attached, bytes carved and number of tables on the
 * current device (each output pointer may be NULL). */
pm_status pm_tables_attach(void* dev_ptr, uint64_t bytes);
pm_status pm_tables_bytes(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                          int32_t elem_bytes, uint64_t* out);
pm_status pm_tables_reset(void);
pm_status pm_tables_info(uint64_t* attached_bytes, uint64_t* used_bytes, int32_t* tables);

/* Workspace bytes pm_mul_u32 / pm_mul_u64 need for this product. */
pm_status pm_workspace_bytes(uint64_t p, int32_t m, int32_t n, int32_t k,
                             int32_t d, int32_t elem_bytes, uint64_t* out);

/* C = A B mod p for uint32 residues (p < 2^32).  A: d*m*n, B: d*n*k,
 * C: (2d-1)*m*k elements, device pointers, 16-byte aligned, C must not
 * overlap A or B.  workspace: device memory of at least
 * pm_workspace_bytes(..., 4, ...) bytes, 256-byte aligned, not overlapping
 * A, B or C; its contents on entry are ignored.  Asynchronous on `stream`. */
pm_status pm_mul_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                     const uint32_t* A, const uint32_t* B, uint32_t* C,
                     void* workspace, uint64_t workspace_bytes, void* stream);

/* Same for uint64 residues, any modulus 2 <= p < 2^62 (CRT mode unless p is
 * an NTT-friendly prime below 2^31). */
pm_status pm_mul_u64(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                     const uint64_t* A, const uint64_t* B, uint64_t* C,
                     void* workspace, uint64_t workspace_bytes, void* stream);

/* pm_mul_u32 (elem_bytes 4) or pm_mul_u64 (elem_bytes 8) without a
 * workspace and without any allocation, for callers that cannot allocate
 * device memory: code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The caller passes only inputs and outputs (same
 * layout, alignment and overlap rules, same result).  The workspace and this
 * entry point's twiddle and Vandermonde tables live in a static device array
 * of 64 MiB that each GPU the library runs on holds until the process ends:
 * 8 MiB of tables and a workspace of at most 56 MiB (58720256 bytes).  A
 * product whose pm_workspace_bytes exceeds that returns PM_ESCRATCH before
 * anything is enqueued; PM_ETABLES if its tables no longer fit the 8 MiB.
 * Calls on one GPU share its array, which keeps the last call's contents
 * (no call relies on them): calls that overlap on one GPU (other streams,
 * other threads) race on the workspace, so the caller serialises them.
 * Asynchronous on `stream`. */
pm_status pm_mul_noalloc(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                         int32_t elem_bytes, const void* A, const void* B, void* C,
                         void* stream);

/* Middle product, and in general a window of coefficients of a product
 * (Section 2, "Polynomial multiplication": MiddleProduct(F, G, c, d) returns
 * the coefficients of degrees c .. c+d-1 of F G for F in K[x]_c and G in
 * K[x]_{c+d}; Section 3, Algorithm PM-Basis, uses its matrix version for the
 * residual).  Here A is an (m x n) matrix with da coefficients (degree < da),
 * B an (n x k) matrix with db coefficients, both coefficient-major as for
 * pm_mul_*, and C receives coefficients lo .. lo+len-1 of A B mod p
 * (len*m*k elements, row c of C = coefficient lo + c).  The paper's
 * MiddleProduct is da = c, db = c + d, lo = c, len = d.  The transform length
 * is the least power of two >= max(da + db - 1 - lo, lo + len): a
 * coefficient of degree >= L that wraps around lands below lo, so the window
 * is exact, and the middle product with c = d costs about half the points of
 * the whole product.  Requires lo >= 0, len >= 1 and lo + len <= da + db - 1
 * (else PM_EINVAL).  Pointer, alignment, overlap and workspace rules and the
 * other status codes are those of pm_mul_*; pm_middle_plan reports the plan
 * and workspace size.  Asynchronous on `stream`. */
pm_status pm_middle_plan(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t da,
                         int32_t db, int32_t lo, int32_t len, int32_t elem_bytes,
                         pm_plan_info* out);
pm_status pm_middle_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t da,
                        int32_t db, int32_t lo, int32_t len, const uint32_t* A,
                        const uint32_t* B, uint32_t* C, void* workspace,
                        uint64_t workspace_bytes, void* stream);
pm_status pm_middle_u64(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t da,
                        int32_t db, int32_t lo, int32_t len, const uint64_t* A,
                        const uint64_t* B, uint64_t* C, void* workspace,
                        uint64_t workspace_bytes, void* stream);

/* C = A B mod p by evaluation at the points 0, 1, ..., 2d-2 and interpolation
 * back, both as matrix products over F_p with (inverse) Vandermonde matrices
 * on the int8 matrix cores (Section 2, "Polynomial matrix multiplication":
 * the adaptation of Doliskani, Giorgi, Lebreton and Schost, which replaces
 * evaluation/interpolation by plain multiplication with Vandermonde
 * matrices, worthwhile for moderate d; and "3-primes" multiplication is not
 * needed for moduli without roots of unity).  Same operands, layout, pointer
 * and workspace rules and result as pm_mul_u32 (workspace size from
 * pm_vdm_workspace_bytes).  Requires p prime, 3 <= p < 2^31, 2d - 1 <= p,
 * 2d - 1 < 4096 and n < 4096 (PM_ERANGE / PM_EINVAL / PM_EUNSUPPORTED
 * otherwise).  The Vandermonde matrices are tables (pm_tables_attach),
 * filled on the device per (p, d) on first use.  Asynchronous on `stream`. */
pm_status pm_vdm_workspace_bytes(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                                 uint64_t* out);
pm_status pm_mul_vdm_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                         const uint32_t* A, const uint32_t* B, uint32_t* C,
                         void* workspace, uint64_t workspace_bytes, void* stream);

/* Evaluation and interpolation at a geometric progression (Section 2,
 * "Polynomial multiplication": with an element a of order at least N, both
 * take O(M(N)) operations; "Polynomial matrix multiplication" uses them for
 * general primes): A and B are evaluated at 1, a, ..., a^(N-1), N = 2d - 1,
 * a the least primitive root of p, the m x n by n x k products are taken at
 * each point, and C is interpolated back.  With C2(t) = t (t - 1) / 2 and
 * i c = C2(i + c) - C2(i) - C2(c), each evaluation is a chirp transform: a
 * middle product of the rows scaled by a^-C2(c) with the fixed polynomial
 * sum a^C2(t) x^t; interpolation is (Q S) mod x^N with Q = prod (x - a^j)
 * and the power series S = sum_i (v_i / Q'(a^i)) / (x - a^i), whose
 * coefficients are another chirp transform.  The four polynomial products
 * run on the transforms of pm_middle_* (modulo word-size NTT primes, since
 * p need not have roots of unity of 2-power order); the tables (chirps,
 * Q, 1/Q'(a^i)) are filled on the device per (p, d) in the table regions.
 * Same layout, pointer, overlap and workspace rules and result as
 * pm_mul_u32 (workspace size from pm_geo_workspace_bytes).  Requires p
 * prime, 3 <= p < 2^31, 2d - 1 <= p - 1 and n < 4096 (PM_ERANGE / PM_EINVAL
 * / PM_EUNSUPPORTED otherwise) and 2(2d - 1) - 1 <= 2^15.  Asynchronous on
 * `stream`. */
pm_status pm_geo_workspace_bytes(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                                 uint64_t* out);
pm_status pm_mul_geo_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                         const uint32_t* A, const uint32_t* B, uint32_t* C,
                         void* workspace, uint64_t workspace_bytes, void* stream);

/* A batch of coefficient windows (pm_middle_* products): each product follows
 * the pm_middle_* rules for its own (m, n, k, da, db, lo, len) and pointers. */
typedef struct pm_window_product {
  int32_t m, n, k, da, db, lo, len, pad;
  const void* A;
  const void* B;
  void* C;
} pm_window_product;

/* Workspace bytes for pm_middle_batched_* over `count` windows (host array). */
pm_status pm_middle_batched_workspace_bytes(uint64_t p, int32_t count,
                                            const pm_window_product* wins,
                                            int32_t elem_bytes, uint64_t* out);

/* All `count` windows in the phase launches of pm_mul_batched_* (as when
 * several independent PM-Basis computations issue their residuals and basis
 * products level by level).  Outputs are identical, byte for byte, to one
 * pm_middle_* call per product.  Asynchronous on `stream`. */
pm_status pm_middle_batched_u32(uint32_t p, int32_t count, const pm_window_product* wins,
                                void* workspace, uint64_t workspace_bytes, void* stream);
pm_status pm_middle_batched_u64(uint64_t p, int32_t count, const pm_window_product* wins,
                                void* workspace, uint64_t workspace_bytes, void* stream);

/* The same M-Basis on the device for `count` instances of one shape at once
 * (one workgroup each), with the same result residue for residue as
 * pm_mbasis_host.  p must be prime (not checked here), 2 <= p < 2^31
 * (PM_ERANGE otherwise).  F: device, instance i at F + i*f_stride
 * (f_stride >= sigma*m*n), residues taken mod p; shift: device, count*m
 * integers; P: device, count*(sigma+1)*m*m residues (instance i at
 * i*(sigma+1)*m*m), overwritten; rdeg: device, count*m integers.
 * workspace: device, at least pm_mbasis_workspace_bytes bytes, 256-byte
 * aligned (PM_EWORKSPACE otherwise).  PM_EUNSUPPORTED when the m x (n + m)
 * elimination matrix does not fit the 160 KiB of LDS (m (n + m) about
 * 40000 at most); PM_EINVAL on sizes < 1 or NULL pointers.  Asynchronous on
 * `stream`. */
pm_status pm_mbasis_workspace_bytes(int32_t count, int32_t m, int32_t n, int32_t sigma,
                                    uint64_t* out);
pm_status pm_mbasis_u32(uint32_t p, int32_t count, int32_t m, int32_t n, int32_t sigma,
                        const uint32_t* F, uint64_t f_stride, const int64_t* shift,
                        uint32_t* P, int64_t* rdeg, void* workspace,
                        uint64_t workspace_bytes, void* stream);

/* Algorithm M-Basis (Section 3, "Approximant bases": sigma rounds of
 * residual, M-Basis-1 returning the s'-Popov basis at order 1, P := Q P and
 * s' := rdeg_s(P)) on the host, for the leaves of PM-Basis, whose polynomial
 * products run through pm_middle_*.  F: host memory, sigma*m*n residues mod
 * p, coefficient-major (coefficient c of entry (i, j) at (c*m + i)*n + j);
 * shift: m host integers.  Output P: host memory of (sigma+1)*m*m residues,
 * coefficient-major, an s-ordered weak Popov approximant basis of (F, sigma)
 * (coefficients above its degree are zero); rdeg_out: m host integers,
 * rdeg_shift(P).  p must be a prime, 2 <= p < 2^62 (PM_EINVAL if not prime,
 * PM_ERANGE if too large); PM_EINVAL on sizes < 1 or NULL pointers;
 * PM_ENOMEM if host memory runs out.  Synchronous; touches no device. */
pm_status pm_mbasis_host(uint64_t p, int32_t m, int32_t n, int32_t sigma,
                         const uint64_t* F, const int64_t* shift, uint64_t* P,
                         int64_t* rdeg_out);

/* Inverse of an n x n matrix mod a prime p < 2^62 on the host (Gauss-Jordan
 * elimination): the constant term A(0)^{-1} that starts Newton iteration for
 * the truncated inverse A^{-1} mod x^N (Section 4, "Lifting techniques").
 * M, Minv: host arrays of n*n residues, row-major.  PM_EINVAL if M is
 * singular mod p, p is not prime, n < 1 or a pointer is NULL; PM_ERANGE if
 * p >= 2^62; PM_ENOMEM if host memory runs out.  Synchronous; touches no
 * device. */
pm_status pm_matinv_host(uint64_t p, int32_t n, const uint64_t* M, uint64_t* Minv);

/* One product of a batch; the pointers follow the pm_mul_* layout rules.
 * A_eval / B_eval: optional evaluations of A / B made by pm_eval_* (NULL:
 * the batch transforms the operand itself).  Given evaluations are used in
 * place of A / B, which are then not read (but must still be valid
 * pointers for the overlap checks). */
typedef struct pm_product {
  int32_t m, n, k, d;
  const void* A;
  const void* B;
  void* C;
  const void* A_eval;
  const void* B_eval;
} pm_product;

/* Evaluations of one operand at the points of the product's transform: the
 * precomputation that the paper's "multiplier classes" keep for repeated
 * products by the same matrix (Section 2, "Polynomial matrix
 * multiplication").  role 0: X is a left operand (rows = m, cols = n);
 * role 1: a right operand (rows = n, cols = k).  X: d*rows*cols residues,
 * coefficient-major, device memory.  The result (X_eval, device memory of at
 * least pm_eval_bytes bytes, 256-byte aligned, owned by the caller) serves
 * every product with the same p, contraction length n and degree bound d,
 * through pm_product.A_eval / B_eval.  Asynchronous on `stream`. */
pm_status pm_eval_bytes(uint64_t p, int32_t role, int32_t rows, int32_t cols, int32_t d,
                        int32_t elem_bytes, uint64_t* out);
pm_status pm_eval_u32(uint32_t p, int32_t role, int32_t rows, int32_t cols, int32_t d,
                      const uint32_t* X, void* X_eval, uint64_t eval_bytes, void* stream);
pm_status pm_eval_u64(uint64_t p, int32_t role, int32_t rows, int32_t cols, int32_t d,
                      const uint64_t* X, void* X_eval, uint64_t eval_bytes, void* stream);

/* Workspace bytes for pm_mul_batched_* over `count` products (host array). */
pm_status pm_batched_workspace_bytes(uint64_t p, int32_t count,
                                     const pm_product* prods, int32_t elem_bytes,
                                     uint64_t* out);

/* All `count` products, each C = A B mod p, in one persistent launch per
 * transform phase set (see the implementation notes in the source).  `prods`
 * is a host array read during the call only.  Outputs are identical, byte
 * for byte, to one pm_mul_* call per product.  Asynchronous on `stream`. */
pm_status pm_mul_batched_u32(uint32_t p, int32_t count, const pm_product* prods,
                             void* workspace, uint64_t workspace_bytes,
                             void* stream);
pm_status pm_mul_batched_u64(uint64_t p, int32_t count, const pm_product* prods,
                             void* workspace, uint64_t workspace_bytes,
                             void* stream);

/* Y = -X mod p elementwise (Y[i] = (p - X[i]) mod p): the negated operand
 * that the Newton iteration for truncated inverses keeps (Section 4,
 * "Lifting techniques": X_2k = X_k - x^k (X_k E mod x^k), computed with -A
 * so that the update is a concatenation).  X, Y: device memory, `count`
 * residues in [0, p) of elem_bytes (4 or 8) bytes, aligned to elem_bytes;
 * Y may equal X (in place), otherwise they must not overlap (PM_EINVAL).
 * p >= 2 and p < 2^32 (elem_bytes 4) or p < 2^62 (elem_bytes 8), else
 * PM_ERANGE.  Asynchronous on `stream`. */
pm_status pm_neg_mod(uint64_t p, const void* X, void* Y, uint64_t count, int32_t elem_bytes,
                     void* stream);

/* Measurement of the VALU issue rate that bounds the transforms (Section 2,
 * "Polynomial multiplication": the butterflies' modular products; here
 * 32-bit high multiplies, the instruction Shoup's products are built from).
 * Launches `blocks` workgroups of 256 threads; each thread runs 8
 * independent chains of `iters` high multiplies, blocks * 256 * iters * 8
 * lane-ops in all, and writes one word to out[blockIdx * 256 + thread]
 * (device memory of at least blocks * 1024 bytes, 4-byte aligned, owned by
 * the caller).  The caller times the launch on `stream` (events around
 * it).  PM_EINVAL for a NULL or misaligned out, blocks outside 1..2^20 or
 * iters 0; PM_EDEVICE if the launch fails.  Asynchronous on `stream`. */
pm_status pm_probe_valu(uint32_t blocks, uint32_t iters, void* out, void* stream);

/* Count the elements of X (count residues of elem_bytes bytes, device
 * memory) that are >= p and write the count to *n_bad (host pointer).  This
 * call synchronises `stream`.  workspace: at least 8 bytes of device memory,
 * 8-byte aligned.  Not on the hot path: an opt-in input check. */
pm_status pm_check_residues(uint64_t p, const void* X, uint64_t count,
                            int32_t elem_bytes, uint64_t* n_bad,
                            void* workspace, void* stream);

/* Kernel timing for measurement.  Between pm_profile_begin and
 * pm_profile_end, every kernel the library launches (from any thread)
 * carries a start and a stop HIP event that its own dispatch fills
 * (hipExtLaunchKernel, on the stream it is launched on), so timing adds no
 * work between kernels; pm_profile_end waits for those events and returns,
 * per kernel kind, the summed device time and the launch count.  Kinds
 * (index into the arrays): 0 forward transform, 1 pointwise products,
 * 2 inverse transform, 3 Chinese remaindering, 5 evaluation and
 * 6 interpolation by Vandermonde products, 7 the row scalings of the
 * geometric-progression products; 4 is a whole batched call of
 * more than two products, timed by an event pair around it (an eager one
 * also reports its phase kernels under 0-3; a replayed graph does not).
 * Launches inside a stream capture are not timed.  Returns PM_EDEVICE if
 * an event could not be created or read; PM_EINVAL if out is NULL. */
#define PM_KERNEL_KINDS 8
typedef struct pm_kernel_stats {
  double total_ms[PM_KERNEL_KINDS];
  uint64_t launches[PM_KERNEL_KINDS];
} pm_kernel_stats;
pm_status pm_profile_begin(void);
pm_status pm_profile_end(pm_kernel_stats* out);
/* Pause (paused != 0) or resume timing inside a pm_profile_begin /
 * pm_profile_end session without dropping what it has recorded, e.g. to
 * time every n-th step of a loop (each timed launch adds a few
 * microseconds of dispatch work).  Returns PM_EINVAL outside a session. */
pm_status pm_profile_pause(int32_t paused);

/* Wait for `stream` and report any device error raised by earlier calls. */
pm_status pm_sync(void* stream);

/* Test hook for the error paths: after `countdown` more host allocation
 * points in the library, the next one fails as if memory ran out (the call
 * then returns PM_ENOMEM); a negative countdown disarms it.  Allocation
 * points are where the library's host code allocates (plans, batch
 * descriptors, table bookkeeping, M-Basis and matrix-inverse work arrays).
 * Process-wide; not for production use. */
pm_status pm_debug_fail_alloc(int32_t countdown);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */
