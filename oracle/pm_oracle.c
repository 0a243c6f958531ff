/*
 * pm_oracle.c -- CPU oracle for polynomial-matrix multiplication over Z/pZ.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, table or header with the GPU
 * library.
 *
 * What it computes (Hyun, Neiger, Schost, ISSAC 2019):
 *   Section 2, "Polynomial multiplication": K[x]_d is the set of polynomials
 *   of degree < d; so an input entry holds d coefficients.
 *   Section 2, "Polynomial matrix multiplication": the product of an (m x n)
 *   and an (n x k) matrix of such polynomials over F_p.  Every variant the
 *   paper lists (evaluation/interpolation at roots of unity or geometric
 *   points, Vandermonde products, the 3-primes lift to Z[x]) computes this
 *   same product, so the oracle is the product's definition written out:
 *
 *     C[c][i][j] = ( sum_{l<n} sum_{a+b=c, 0<=a,b<d} A[a][i][l] * B[b][l][j] ) mod p
 *
 *   for 0 <= c <= 2d-2, 0 <= i < m, 0 <= j < k.  Storage is coefficient-major:
 *   element (c, i, j) of an R x S matrix is at offset (c*R + i)*S + j.
 *
 * Arithmetic: exact.  Products of residues < 2^62 are accumulated in unsigned
 * 128-bit integers and reduced mod p before the accumulator can overflow.
 * Inputs are reduced mod p on entry so the function is defined on any input.
 *
 * Checkers used at sizes where the full schoolbook is too slow:
 *   orc_eval_at      -- Horner evaluation of every entry at one point r
 *                       (C(r) = A(r) B(r) is the evaluation homomorphism).
 *   orc_project_*    -- u^T X(x) v projections (Freivalds) on coefficients.
 *   orc_polymul      -- plain univariate schoolbook product mod p.
 *   orc_is_prime     -- deterministic Miller-Rabin for 64-bit integers.
 *
 * Planted mistakes for mutation tests are compiled in only with -DORC_PLANT=n
 * (see the switch below); the default build has none.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

/* ---- scalar helpers ---------------------------------------------------- */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) {
    return (uint64_t)(((u128)a * b) % p);
}

uint64_t orc_powmod(uint64_t b, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    b %= p;
    while (e) {
        if (e & 1) r = mulmod(r, b, p);
        b = mulmod(b, b, p);
        e >>= 1;
    }
    return r;
}

/* Deterministic Miller-Rabin: the first twelve primes as bases are enough for
 * every n < 3.18e23, hence for all 64-bit n. */
int orc_is_prime(uint64_t n) {
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int t = 0; t < 12; ++t) {
        if (n % bases[t] == 0) return n == bases[t];
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (int t = 0; t < 12; ++t) {
        uint64_t x = orc_powmod(bases[t], d, n);
        if (x == 1 || x == n - 1) continue;
        int witness = 1;
        for (int r = 1; r < s; ++r) {
            x = mulmod(x, x, n);
            if (x == n - 1) { witness = 0; break; }
        }
        if (witness) return 0;
    }
    return 1;
}

/* Largest number of products (p-1)^2 that can be added to a value < p in an
 * unsigned 128-bit accumulator without overflow. */
static uint64_t safe_terms(uint64_t p) {
    u128 sq = (u128)(p - 1) * (p - 1);
    if (sq == 0) return UINT64_MAX;
    u128 room = ~(u128)0 - (p - 1);
    u128 t = room / sq;
    return t > (u128)UINT64_MAX ? UINT64_MAX : (uint64_t)t;
}

/* ---- univariate schoolbook product -------------------------------------- */

/* out[0 .. la+lb-2] = (a * b) mod p, a has la coefficients, b has lb. */
void orc_polymul(uint64_t p, int la, const uint64_t* a, int lb, const uint64_t* b,
                 uint64_t* out) {
    const uint64_t lim = safe_terms(p);
    for (int c = 0; c <= la + lb - 2; ++c) {
        int lo = c - (lb - 1) > 0 ? c - (lb - 1) : 0;
        int hi = c < la - 1 ? c : la - 1;
        u128 acc = 0;
        uint64_t cnt = 0;
        for (int x = lo; x <= hi; ++x) {
            acc += (u128)(a[x] % p) * (b[c - x] % p);
            if (++cnt == lim) { acc %= p; cnt = 0; }
        }
        out[c] = (uint64_t)(acc % p);
    }
}

/* ---- one output entry of the polynomial-matrix product ------------------ */

typedef struct {
    uint64_t p;
    int m, n, k, d;
    const uint64_t* A;
    const uint64_t* B;
} prob_t;

/* All 2d-1 coefficients of C_ij = sum_l A_il * B_lj, written to out[c].
 * ga and gb hold n*d gathered coefficients each: ga[l*d + a] = A[a][i][l],
 * gb[l*d + b] = B[b][l][j]. */
static void entry(const prob_t* P, int i, int j, uint64_t* out, uint64_t* ga,
                  uint64_t* gb) {
    const uint64_t p = P->p;
    const int m = P->m, n = P->n, k = P->k, d = P->d;
    const uint64_t lim = safe_terms(p);
    const int len = 2 * d - 1;
    for (int l = 0; l < n; ++l) {
        for (int a = 0; a < d; ++a) {
            ga[(size_t)l * d + a] = P->A[((size_t)a * m + i) * n + l] % p;
#if ORC_PLANT == 2
            /* planted: B read transposed (entry (j, l) instead of (l, j)) */
            gb[(size_t)l * d + a] = P->B[((size_t)a * n + (j % n)) * k + (l % k)] % p;
#else
            gb[(size_t)l * d + a] = P->B[((size_t)a * n + l) * k + j] % p;
#endif
        }
    }
    for (int c = 0; c < len; ++c) {
        /* coefficient c collects A[a] * B[c - a] for max(0, c-d+1) <= a <= min(c, d-1) */
        const int lo = c - (d - 1) > 0 ? c - (d - 1) : 0;
#if ORC_PLANT == 1
        /* planted: the last term of every convolution sum is dropped */
        const int hi = (c < d - 1 ? c : d - 1) - 1;
#else
        const int hi = c < d - 1 ? c : d - 1;
#endif
        u128 acc = 0;
        uint64_t cnt = 0;
        for (int l = 0; l < n; ++l) {
            const uint64_t* fa = ga + (size_t)l * d;
#if ORC_PLANT == 3
            /* planted: B's index is off by one */
            const uint64_t* fb = gb + (size_t)l * d + 1;
#else
            const uint64_t* fb = gb + (size_t)l * d;
#endif
            int a = lo;
            while (a <= hi) {
                uint64_t room = lim - cnt;
                int stop = hi;
                if ((uint64_t)(hi - a + 1) > room) stop = a + (int)room - 1;
                for (int x = a; x <= stop; ++x) acc += (u128)fa[x] * fb[c - x];
                cnt += (uint64_t)(stop - a + 1);
#if ORC_PLANT == 4
                /* planted: the reduction is skipped, so the accumulator overflows */
                if (cnt == lim) { cnt = 0; }
#else
                if (cnt == lim) { acc %= p; cnt = 0; }
#endif
                a = stop + 1;
            }
        }
#if ORC_PLANT == 5
        /* planted: result reduced mod p-1 */
        out[c] = (uint64_t)(acc % (p - 1 ? p - 1 : 1));
#else
        out[c] = (uint64_t)(acc % p);
#endif
    }
}

typedef struct {
    const prob_t* P;
    int count;             /* entries to compute */
    const int32_t* ii;     /* row of entry s, or NULL: entry s = (s / k, s % k) */
    const int32_t* jj;
    uint64_t* out;         /* entry s -> out[s * (2d-1) .. ] or full C if full */
    int full;              /* 1: write coefficient-major C, 0: per-entry rows */
    int next;              /* shared work counter */
    pthread_mutex_t lock;
} job_t;

static void* worker(void* arg) {
    job_t* J = (job_t*)arg;
    const prob_t* P = J->P;
    const int len = 2 * P->d - 1;
    uint64_t* ga = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)P->n * P->d + 8);
    uint64_t* gb = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)P->n * P->d + 8);
    uint64_t* row = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)len);
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int s = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (s >= J->count) break;
        int i = J->ii ? J->ii[s] : s / P->k;
        int j = J->jj ? J->jj[s] : s % P->k;
        entry(P, i, j, row, ga, gb);
        if (J->full) {
            for (int c = 0; c < len; ++c)
                J->out[((size_t)c * P->m + i) * P->k + j] = row[c];
        } else {
            memcpy(J->out + (size_t)s * len, row, sizeof(uint64_t) * (size_t)len);
        }
    }
    free(ga); free(gb); free(row);
    return NULL;
}

static int run(job_t* J, int threads) {
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    pthread_mutex_init(&J->lock, NULL);
    J->next = 0;
    int started = 0;
    for (int t = 0; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, worker, J) == 0) ++started;
    }
    if (started == 0) worker(J);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    pthread_mutex_destroy(&J->lock);
    return 0;
}

static int bad_args(uint64_t p, int m, int n, int k, int d) {
    return p < 2 || p >= (1ULL << 63) || m < 1 || n < 1 || k < 1 || d < 1;
}

/* Full product: C has (2d-1) x m x k coefficients, coefficient-major. */
int orc_polymatmul(uint64_t p, int m, int n, int k, int d, const uint64_t* A,
                   const uint64_t* B, uint64_t* C, int threads) {
    if (bad_args(p, m, n, k, d)) return -1;
    prob_t P = {p, m, n, k, d, A, B};
    job_t J;
    memset(&J, 0, sizeof J);
    J.P = &P; J.count = m * k; J.out = C; J.full = 1;
    return run(&J, threads);
}

/* Selected entries: out[s*(2d-1) + c] = C[c][ii[s]][jj[s]]. */
int orc_polymatmul_entries(uint64_t p, int m, int n, int k, int d,
                           const uint64_t* A, const uint64_t* B, int count,
                           const int32_t* ii, const int32_t* jj, uint64_t* out,
                           int threads) {
    if (bad_args(p, m, n, k, d) || count < 0) return -1;
    for (int s = 0; s < count; ++s) {
        if (ii[s] < 0 || ii[s] >= m || jj[s] < 0 || jj[s] >= k) return -1;
    }
    prob_t P = {p, m, n, k, d, A, B};
    job_t J;
    memset(&J, 0, sizeof J);
    J.P = &P; J.count = count; J.ii = ii; J.jj = jj; J.out = out; J.full = 0;
    return run(&J, threads);
}

/* ---- checkers ------------------------------------------------------------ */

/* Work split for the checkers: item ranges [lo, hi) handed out to threads. */
typedef struct {
    void (*fn)(void* ctx, size_t lo, size_t hi);
    void* ctx;
    size_t count, chunk, next;
    pthread_mutex_t lock;
} split_t;

static void* split_worker(void* arg) {
    split_t* S = (split_t*)arg;
    for (;;) {
        pthread_mutex_lock(&S->lock);
        size_t lo = S->next;
        S->next = lo + S->chunk < S->count ? lo + S->chunk : S->count;
        size_t hi = S->next;
        pthread_mutex_unlock(&S->lock);
        if (lo >= hi) break;
        S->fn(S->ctx, lo, hi);
    }
    return NULL;
}

static void split_run(void (*fn)(void*, size_t, size_t), void* ctx, size_t count,
                      size_t chunk, int threads) {
    split_t S;
    S.fn = fn; S.ctx = ctx; S.count = count; S.chunk = chunk ? chunk : 1; S.next = 0;
    pthread_mutex_init(&S.lock, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[t], NULL, split_worker, &S) == 0) ++started;
    if (started == 0) split_worker(&S);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    pthread_mutex_destroy(&S.lock);
}

/* Horner evaluation of every entry at several points. */
typedef struct {
    uint64_t p;
    size_t rc;             /* entries (rows * cols) */
    int deg, npts;
    const uint64_t* X;     /* (deg, rows, cols) coefficient-major */
    const uint64_t* pts;   /* npts points, reduced mod p */
    uint64_t* out;         /* out[t * rc + e] = X_e(pts[t]) */
} eval_t;

static void eval_range(void* ctx, size_t lo, size_t hi) {
    const eval_t* E = (const eval_t*)ctx;
    const uint64_t p = E->p;
    for (int t = 0; t < E->npts; ++t) {
        const uint64_t r = E->pts[t];
        uint64_t* o = E->out + (size_t)t * E->rc;
        for (size_t e = lo; e < hi; ++e) o[e] = 0;
        for (int c = E->deg - 1; c >= 0; --c) {
            const uint64_t* row = E->X + (size_t)c * E->rc;
            if (p <= 0xFFFFFFFFull) {
                /* o r + x <= (p-1)^2 + (p-1) < 2^64 */
                for (size_t e = lo; e < hi; ++e) o[e] = (o[e] * r + row[e] % p) % p;
            } else {
                for (size_t e = lo; e < hi; ++e)
                    o[e] = (uint64_t)(((u128)o[e] * r + row[e] % p) % p);
            }
        }
    }
}

/* out[t*rows*cols + i*cols + j] = X_ij(pts[t]) mod p, X stored (deg, rows, cols)
 * coefficient-major; Horner's rule from the top coefficient down. */
void orc_eval_points(uint64_t p, int rows, int cols, int deg, const uint64_t* X, int npts,
                     const uint64_t* pts, uint64_t* out, int threads) {
    uint64_t* r = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(npts > 0 ? npts : 1));
    for (int t = 0; t < npts; ++t) r[t] = pts[t] % p;
    eval_t E = {p, (size_t)rows * cols, deg, npts, X, r, out};
    split_run(eval_range, &E, E.rc, 4096, threads);
    free(r);
}

void orc_eval_at(uint64_t p, int rows, int cols, int deg, const uint64_t* X,
                 uint64_t r, uint64_t* out) {
    orc_eval_points(p, rows, cols, deg, X, 1, &r, out, 1);
}

/* Plain matrix product mod p: Z (m x k) = X (m x n) * Y (n x k), row-major. */
void orc_matmul(uint64_t p, int m, int n, int k, const uint64_t* X,
                const uint64_t* Y, uint64_t* Z) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < k; ++j) {
            u128 acc = 0;
            for (int l = 0; l < n; ++l)
                acc = (acc + (u128)(X[(size_t)i * n + l] % p) * (Y[(size_t)l * k + j] % p)) % p;
            Z[(size_t)i * k + j] = (uint64_t)acc;
        }
}

/* Projections over the coefficients c of a (deg, rows, cols) matrix. */
typedef struct {
    uint64_t p;
    int rows, cols, left;
    const uint64_t* X;
    const uint64_t* w;     /* u (rows) for left, v (cols) for right; reduced mod p */
    uint64_t* out;         /* left: (deg, cols); right: (deg, rows) */
} proj_t;

static void proj_range(void* ctx, size_t lo, size_t hi) {
    const proj_t* P = (const proj_t*)ctx;
    const uint64_t p = P->p, lim = safe_terms(p);
    const int rows = P->rows, cols = P->cols;
    const int width = P->left ? cols : rows;
    u128* acc = (u128*)malloc(sizeof(u128) * (size_t)width);
    for (size_t c = lo; c < hi; ++c) {
        const uint64_t* Xc = P->X + c * (size_t)rows * cols;
        for (int t = 0; t < width; ++t) acc[t] = 0;
        if (P->left) {
            /* out[c][col] = sum_row u[row] X[c][row][col] */
            uint64_t cnt = 0;
            for (int row = 0; row < rows; ++row) {
                const uint64_t ur = P->w[row];
                for (int col = 0; col < cols; ++col)
                    acc[col] += (u128)ur * (Xc[(size_t)row * cols + col] % p);
                if (++cnt == lim) {
                    for (int col = 0; col < cols; ++col) acc[col] %= p;
                    cnt = 0;
                }
            }
        } else {
            /* out[c][row] = sum_col X[c][row][col] v[col] */
            for (int row = 0; row < rows; ++row) {
                u128 a = 0;
                uint64_t cnt = 0;
                for (int col = 0; col < cols; ++col) {
                    a += (u128)(Xc[(size_t)row * cols + col] % p) * P->w[col];
                    if (++cnt == lim) { a %= p; cnt = 0; }
                }
                acc[row] = a;
            }
        }
        for (int t = 0; t < width; ++t) P->out[c * (size_t)width + t] = (uint64_t)(acc[t] % p);
    }
    free(acc);
}

static void project(uint64_t p, int rows, int cols, int deg, const uint64_t* X,
                    const uint64_t* w, uint64_t* out, int left, int threads) {
    const int width = left ? rows : cols;
    uint64_t* wr = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(width > 0 ? width : 1));
    for (int t = 0; t < width; ++t) wr[t] = w[t] % p;
    proj_t P = {p, rows, cols, left, X, wr, out};
    split_run(proj_range, &P, (size_t)deg, 16, threads);
    free(wr);
}

/* Left projection: out[c][col] = sum_row u[row] * X[c][row][col] mod p. */
void orc_project_left(uint64_t p, int rows, int cols, int deg, const uint64_t* X,
                      const uint64_t* u, uint64_t* out) {
    project(p, rows, cols, deg, X, u, out, 1, 1);
}

/* Right projection: out[c][row] = sum_col X[c][row][col] * v[col] mod p. */
void orc_project_right(uint64_t p, int rows, int cols, int deg, const uint64_t* X,
                       const uint64_t* v, uint64_t* out) {
    project(p, rows, cols, deg, X, v, out, 0, 1);
}

/* Threaded forms of the two projections. */
void orc_project_left_mt(uint64_t p, int rows, int cols, int deg, const uint64_t* X,
                         const uint64_t* u, uint64_t* out, int threads) {
    project(p, rows, cols, deg, X, u, out, 1, threads);
}

void orc_project_right_mt(uint64_t p, int rows, int cols, int deg, const uint64_t* X,
                          const uint64_t* v, uint64_t* out, int threads) {
    project(p, rows, cols, deg, X, v, out, 0, threads);
}

/* Sum of n univariate schoolbook products: out[c] = sum_l sum_{a+b=c} U[l][a] V[l][b]
 * mod p, U and V holding n polynomials of d coefficients each (row l at l*d),
 * for 0 <= c <= 2d-2; threads split the output coefficients. */
typedef struct {
    uint64_t p;
    int n, d;
    const uint64_t* U;
    const uint64_t* V;
    uint64_t* out;
} psum_t;

static void psum_range(void* ctx, size_t lo, size_t hi) {
    const psum_t* S = (const psum_t*)ctx;
    const uint64_t p = S->p, lim = safe_terms(p);
    const int d = S->d;
    for (size_t cc = lo; cc < hi; ++cc) {
        const int c = (int)cc;
        const int a0 = c - (d - 1) > 0 ? c - (d - 1) : 0;
        const int a1 = c < d - 1 ? c : d - 1;
        u128 acc = 0;
        uint64_t cnt = 0;
        for (int l = 0; l < S->n; ++l) {
            const uint64_t* u = S->U + (size_t)l * d;
            const uint64_t* v = S->V + (size_t)l * d;
            for (int a = a0; a <= a1; ++a) {
                acc += (u128)u[a] * v[c - a];
                if (++cnt == lim) { acc %= p; cnt = 0; }
            }
        }
        S->out[c] = (uint64_t)(acc % p);
    }
}

void orc_polymul_sum(uint64_t p, int n, int d, const uint64_t* U, const uint64_t* V,
                     uint64_t* out, int threads) {
    const size_t len = (size_t)n * d;
    uint64_t* u = (uint64_t*)malloc(sizeof(uint64_t) * (len ? len : 1));
    uint64_t* v = (uint64_t*)malloc(sizeof(uint64_t) * (len ? len : 1));
    for (size_t t = 0; t < len; ++t) { u[t] = U[t] % p; v[t] = V[t] % p; }
    psum_t S = {p, n, d, u, v, out};
    split_run(psum_range, &S, (size_t)(2 * d - 1), 8, threads);
    free(u); free(v);
}
