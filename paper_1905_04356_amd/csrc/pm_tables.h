// pm_tables.h -- device tables (roots of unity with their Shoup companions,
// Vandermonde matrices) in device memory that the caller owns.
//
// The caller registers one or more regions per device (pm_tables_attach).
// A table is carved from them the first time a call needs it and filled by a
// kernel on that call's stream; nothing is copied from the host and the
// library allocates no device memory.  Later calls reuse it.  A table first
// filled inside a stream capture is filled again by the captured graph on
// every replay, and by the next eager call that needs it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_plan.h"

namespace pm {

// One (prime, transform length, pass structure) whose twiddle tables a
// launch reads.
struct TwKey {
  uint32_t q;
  int logL, split, maxr;
};

// Bytes of the forward and inverse twiddle tables for a length-2^logL
// transform with the pass structure make_pass_plan(logL, split, maxr),
// 256-byte aligned.
uint64_t twiddle_table_bytes(int logL, int split, int maxr);
// Bytes of the Vandermonde tables for degree bound d (V, W and the helper
// arrays they are built from), 256-byte aligned.
uint64_t vdm_table_bytes(int d);

// Make the twiddle tables of keys[0 .. n) available to work enqueued on s
// after this call: carve and fill missing ones, make s wait for fills
// enqueued on another stream that may still run.  All or nothing: if the
// regions cannot hold every missing table, nothing is carved or enqueued and
// PM_ETABLES is returned.  PM_EDEVICE if a launch fails.
int prepare_twiddles(const TwKey* keys, int n, hipStream_t s);

// Constants and device table pointers of a prepared key; PM_EINVAL if the
// key was never prepared on the current device.
int prime_const(const TwKey& key, PrimeConst* out);

// Host part of PrimeConst (q, L^-1 and its companion, Barrett constant).
void prime_const_host(uint32_t q, int logL, PrimeConst* out);
// Primitive 2^logL-th root of unity mod q (0 if none).
uint32_t root_of_unity(uint32_t q, int logL);

// Vandermonde tables for evaluation at 0 .. 2d-2 mod p and interpolation
// back: prepared like the twiddle tables.
int prepare_vdm(uint32_t p, int d, hipStream_t s, const uint32_t** V, const uint32_t** W);

// Tables of the evaluation/interpolation at the geometric progression
// a^0 .. a^(N-1) mod p (N = 2d - 1, a the least primitive root of p):
// spos[t] = a^C2(t) and sneg[t] = a^-C2(t) for t < T = 2N - 1, with
// C2(t) = t (t - 1) / 2; nspos[t] = -a^C2(t) and fc[t] = a^(C2(t) - t) /
// Q'(a^t) for t < N; q: the N + 1 coefficients of Q(x) = prod_j (x - a^j).
struct GeoTables {
  uint32_t p, a, N, T;
  uint32_t *spos, *sneg, *nspos, *fc, *q;
};
uint64_t geo_table_bytes(int d);
// Prepared like the twiddle tables; PM_EUNSUPPORTED if p has no element of
// order at least N (p - 1 < N).
int prepare_geo(uint32_t p, int d, hipStream_t s, GeoTables* out);
int launch_fill_geo(const GeoTables& g, hipStream_t s);
// Y[r] = X[src] f[src] mod p row by row (src = r, or rows - 1 - r when
// reverse), rows of E residues.
int launch_geo_scale(const uint32_t* X, uint32_t* Y, uint32_t rows, uint64_t E,
                     const uint32_t* f, int reverse, uint32_t p, hipStream_t s);

// Table pools: the regions the caller registers (pm_tables_attach), and the
// slice of the static scratch array that the no-allocation entry point keeps
// its tables in.  A TablePool scope selects the pool of this thread's calls.
constexpr int kPoolCaller = 0, kPoolStatic = 1;
class TablePool {
 public:
  explicit TablePool(int pool);
  ~TablePool();
  TablePool(const TablePool&) = delete;
  TablePool& operator=(const TablePool&) = delete;

 private:
  int prev_;
};
// Register a region of device memory in `pool` on the current device.
int tables_attach_pool(int pool, void* dev_ptr, uint64_t bytes);

// Incremented by pm_tables_reset: table pointers recorded under an older
// epoch (in captured graphs) are stale.
uint64_t tables_epoch();

// Device fills (pm_tables.hip).  dst holds max(tw_count, 1) forward entries
// followed by as many inverse ones.
int launch_fill_twiddles(const TwKey& key, uint32_t w, uint32_t winv, Tw* dst, hipStream_t s);
// V: (2d-1) x d, W: (2d-1) x (2d-1), work: 2(2d-1) + 1 words of helper data.
int launch_fill_vdm(uint32_t p, int d, uint32_t* V, uint32_t* W, uint32_t* work,
                    hipStream_t s);

}  // namespace pm
