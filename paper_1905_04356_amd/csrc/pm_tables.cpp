// pm_tables.cpp -- bookkeeping of the device tables that live in regions of
// caller-owned device memory (pm_tables_attach): carving, fills on the
// caller's stream, ordering between streams, stream capture.
#include "pm_tables.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/pm.h"

namespace pm {

namespace {

// kind 0: twiddles (a = q, b = logL, c = pass structure: split, maxr);
// kind 1: Vandermonde (a = p, b = d); kind 2: geometric progression (a = p,
// b = d).
typedef std::tuple<int, uint32_t, int, uint64_t> Key;

enum FillState {
  kCapturedOnly = 0,  // filled only inside a capture: eager users fill it again
  kPending = 1,       // filled eagerly on `stream`; `ev` marks its end
  kReady = 2          // that fill is known to have completed
};

struct Entry {
  uint8_t* ptr = nullptr;
  int state = kCapturedOnly;
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;
};

struct Region {
  uint8_t* base;
  uint64_t bytes, used;
};

struct DevTables {
  std::vector<Region> regions;
  std::map<Key, Entry> entries;
};

std::mutex g_mu;
std::map<int, DevTables> g_dev;  // keyed by pool_key(pool, device)
std::atomic<uint64_t> g_epoch{0};
thread_local int t_pool = kPoolCaller;

int pool_key(int pool, int dev) { return pool * 4096 + dev; }

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

uint64_t pass_signature(const TwKey& k) { return (uint64_t)k.split * 16 + (uint64_t)k.maxr; }

// Carve `bytes` from the device's regions (first fit, bump allocation).
uint8_t* carve(DevTables& D, uint64_t bytes) {
  for (Region& r : D.regions) {
    const uint64_t at = align_up(r.used, 256);
    if (at + bytes <= r.bytes) {
      r.used = at + bytes;
      return r.base + at;
    }
  }
  return nullptr;
}

struct Want {
  Key key;
  uint64_t bytes;
};

// Shared logic of prepare_twiddles / prepare_vdm: make every wanted entry
// usable on s; `fill(key, ptr)` enqueues one fill on s.
template <typename Fill>
int prepare(const std::vector<Want>& want, hipStream_t s, Fill fill,
            std::vector<uint8_t*>* ptrs) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PM_EDEVICE;
  const bool capturing = stream_capturing(s);
  std::lock_guard<std::mutex> lock(g_mu);
  DevTables& D = g_dev[pool_key(t_pool, dev)];
  // 1. carve every missing entry, all or nothing
  std::vector<Region> saved = D.regions;
  std::vector<Key> added;
  for (const Want& w : want) {
    if (D.entries.count(w.key)) continue;
    uint8_t* p = carve(D, w.bytes);
    if (!p) {
      D.regions = saved;
      for (const Key& k : added) D.entries.erase(k);
      return PM_ETABLES;
    }
    Entry e;
    e.ptr = p;
    e.state = -1;  // new: filled below
    D.entries.emplace(w.key, e);
    added.push_back(w.key);
  }
  // 2. fills and waits
  ptrs->clear();
  for (const Want& w : want) {
    Entry& e = D.entries[w.key];
    ptrs->push_back(e.ptr);
    if (e.state == kReady) continue;
    if (e.state == kPending && !capturing) {
      const hipError_t q = hipEventQuery(e.ev);
      if (q == hipSuccess) {
        e.state = kReady;
        continue;
      }
      if (q != hipErrorNotReady) return PM_EDEVICE;
      if (e.stream != s && hipStreamWaitEvent(s, e.ev, 0) != hipSuccess) return PM_EDEVICE;
      continue;
    }
    // new, filled only in a capture, or (inside a capture) not known to be
    // complete: fill it on s.  Refilling writes the same values.
    if (fill(w.key, e.ptr) != hipSuccess) return PM_EDEVICE;
    if (capturing) {
      if (e.state == -1) e.state = kCapturedOnly;
      continue;
    }
    if (!e.ev && hipEventCreateWithFlags(&e.ev, hipEventDisableTiming) != hipSuccess) {
      e.ev = nullptr;
      return PM_EDEVICE;
    }
    if (hipEventRecord(e.ev, s) != hipSuccess) return PM_EDEVICE;
    e.state = kPending;
    e.stream = s;
  }
  return PM_OK;
}

uint32_t shoup_of(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

// Smallest generator of (Z/qZ)^*.
uint32_t primitive_root(uint32_t q) {
  std::vector<uint64_t> f;
  uint64_t x = q - 1;
  for (uint64_t t = 2; t * t <= x; ++t) {
    if (x % t == 0) {
      f.push_back(t);
      while (x % t == 0) x /= t;
    }
  }
  if (x > 1) f.push_back(x);
  for (uint32_t g = 2; g < q; ++g) {
    bool ok = true;
    for (uint64_t t : f)
      if (powmod_u64(g, (q - 1) / t, q) == 1) { ok = false; break; }
    if (ok) return g;
  }
  return 0;
}

}  // namespace

uint64_t tables_epoch() { return g_epoch.load(); }

TablePool::TablePool(int pool) : prev_(t_pool) { t_pool = pool; }
TablePool::~TablePool() { t_pool = prev_; }

int tables_attach_pool(int pool, void* dev_ptr, uint64_t bytes) {
  if (!dev_ptr || ((uintptr_t)dev_ptr & 255) || bytes < 256) return PM_EINVAL;
  try {
    alloc_point();  // the region list and the device's table map
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PM_EDEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    DevTables& D = g_dev[pool_key(pool, dev)];
    for (const Region& r : D.regions) {
      const uintptr_t a = (uintptr_t)r.base, b = (uintptr_t)dev_ptr;
      if (a < b + bytes && b < a + r.bytes) return PM_EINVAL;  // overlaps a region
    }
    D.regions.push_back(Region{(uint8_t*)dev_ptr, bytes, 0});
    return PM_OK;
  } catch (const std::bad_alloc&) {
    return PM_ENOMEM;
  }
}

uint64_t twiddle_table_bytes(int logL, int split, int maxr) {
  const PassPlan PP = make_pass_plan(logL, split, maxr);
  const uint64_t cnt = PP.tw_count ? PP.tw_count : 1;
  return align_up(2 * cnt * sizeof(Tw), 256);
}

uint64_t vdm_table_bytes(int d) {
  const uint64_t N = 2ull * d - 1;
  return align_up(4 * N * d, 256) + align_up(4 * N * N, 256) + align_up(4 * (2 * N + 1), 256);
}

uint32_t root_of_unity(uint32_t q, int logL) {
  static std::mutex mu;
  static std::map<uint32_t, uint32_t> gens;
  if (q < 3 || v2_u64(q - 1) < logL) return 0;
  uint32_t g;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = gens.find(q);
    if (it == gens.end()) it = gens.emplace(q, primitive_root(q)).first;
    g = it->second;
  }
  if (g == 0) return 0;
  return (uint32_t)powmod_u64(g, (q - 1) >> logL, q);
}

void prime_const_host(uint32_t q, int logL, PrimeConst* out) {
  memset(out, 0, sizeof *out);
  const uint64_t L = 1ull << logL;
  out->q = q;
  out->linv = (uint32_t)powmod_u64(L % q, q - 2, q);
  out->linv_p = shoup_of(out->linv, q);
  out->mu = ~0ull / q;
  if (logL >= 2) {
    out->i4 = (uint32_t)powmod_u64(root_of_unity(q, logL), L / 4, q);
    out->i4p = shoup_of(out->i4, q);
  }
}

int prepare_twiddles(const TwKey* keys, int n, hipStream_t s) {
  try {
    alloc_point();  // the key list here, the table map and regions in prepare()
    std::vector<Want> want;
    for (int i = 0; i < n; ++i) {
      const Key k(0, keys[i].q, keys[i].logL, pass_signature(keys[i]));
      bool dup = false;
      for (const Want& w : want) dup = dup || w.key == k;
      if (dup) continue;
      if (!root_of_unity(keys[i].q, keys[i].logL)) return PM_EUNSUPPORTED;
      want.push_back(Want{k, twiddle_table_bytes(keys[i].logL, keys[i].split, keys[i].maxr)});
    }
    std::vector<uint8_t*> ptrs;
    return prepare(
        want, s,
        [&](const Key& k, uint8_t* p) {
          const uint64_t sig = std::get<3>(k);
          const TwKey key{std::get<1>(k), std::get<2>(k), (int)(sig / 16), (int)(sig % 16)};
          const uint32_t w = root_of_unity(key.q, key.logL);
          const uint32_t winv = (uint32_t)powmod_u64(w, (1ull << key.logL) - 1, key.q);
          return launch_fill_twiddles(key, w, winv, (Tw*)p, s);
        },
        &ptrs);
  } catch (const std::bad_alloc&) {
    return PM_ENOMEM;
  }
}

int prime_const(const TwKey& key, PrimeConst* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PM_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  auto d = g_dev.find(pool_key(t_pool, dev));
  if (d == g_dev.end()) return PM_EINVAL;
  auto it = d->second.entries.find(Key(0, key.q, key.logL, pass_signature(key)));
  if (it == d->second.entries.end()) return PM_EINVAL;
  prime_const_host(key.q, key.logL, out);
  const PassPlan PP = make_pass_plan(key.logL, key.split, key.maxr);
  const size_t cnt = PP.tw_count ? PP.tw_count : 1;
  out->tw_fwd = (const Tw*)it->second.ptr;
  out->tw_inv = (const Tw*)it->second.ptr + cnt;
  return PM_OK;
}

int prepare_vdm(uint32_t p, int d, hipStream_t s, const uint32_t** V, const uint32_t** W) {
  try {
    alloc_point();  // as in prepare_twiddles
    const uint64_t N = 2ull * d - 1;
    std::vector<Want> want{Want{Key(1, p, d, 0), vdm_table_bytes(d)}};
    auto split = [&](uint8_t* base, uint32_t** v, uint32_t** w, uint32_t** work) {
      *v = (uint32_t*)base;
      *w = (uint32_t*)(base + align_up(4 * N * d, 256));
      *work = (uint32_t*)(base + align_up(4 * N * d, 256) + align_up(4 * N * N, 256));
    };
    std::vector<uint8_t*> ptrs;
    const int st = prepare(
        want, s,
        [&](const Key&, uint8_t* base) {
          uint32_t *v, *w, *work;
          split(base, &v, &w, &work);
          return launch_fill_vdm(p, d, v, w, work, s);
        },
        &ptrs);
    if (st != PM_OK) return st;
    uint32_t *v, *w, *work;
    split(ptrs[0], &v, &w, &work);
    *V = v;
    *W = w;
    return PM_OK;
  } catch (const std::bad_alloc&) {
    return PM_ENOMEM;
  }
}

uint64_t geo_table_bytes(int d) {
  const uint64_t N = 2ull * d - 1, T = 2 * N - 1;
  return 2 * align_up(4 * T, 256) + 2 * align_up(4 * N, 256) + align_up(4 * (N + 1), 256);
}

int prepare_geo(uint32_t p, int d, hipStream_t s, GeoTables* out) {
  try {
    alloc_point();  // as in prepare_twiddles
    const uint32_t N = 2u * (uint32_t)d - 1, T = 2 * N - 1;
    if (p < 3 || (uint64_t)N > (uint64_t)p - 1) return PM_EUNSUPPORTED;
    const uint32_t a = primitive_root(p);
    if (!a) return PM_EUNSUPPORTED;
    std::vector<Want> want{Want{Key(2, p, d, 0), geo_table_bytes(d)}};
    auto split = [&](uint8_t* base, GeoTables* g) {
      g->p = p; g->a = a; g->N = N; g->T = T;
      uint64_t off = 0;
      g->spos = (uint32_t*)(base + off); off += align_up(4ull * T, 256);
      g->sneg = (uint32_t*)(base + off); off += align_up(4ull * T, 256);
      g->nspos = (uint32_t*)(base + off); off += align_up(4ull * N, 256);
      g->fc = (uint32_t*)(base + off); off += align_up(4ull * N, 256);
      g->q = (uint32_t*)(base + off);
    };
    std::vector<uint8_t*> ptrs;
    const int st = prepare(
        want, s,
        [&](const Key&, uint8_t* base) {
          GeoTables g;
          split(base, &g);
          return launch_fill_geo(g, s);
        },
        &ptrs);
    if (st != PM_OK) return st;
    split(ptrs[0], out);
    return PM_OK;
  } catch (const std::bad_alloc&) {
    return PM_ENOMEM;
  }
}

}  // namespace pm

extern "C" {

pm_status pm_tables_attach(void* dev_ptr, uint64_t bytes) {
  return (pm_status)pm::tables_attach_pool(pm::kPoolCaller, dev_ptr, bytes);
}

pm_status pm_tables_reset(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PM_EDEVICE;
  std::lock_guard<std::mutex> lock(pm::g_mu);
  auto it = pm::g_dev.find(pm::pool_key(pm::kPoolCaller, dev));
  if (it == pm::g_dev.end()) return PM_OK;
  for (auto& kv : it->second.entries)
    if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
  pm::g_dev.erase(it);
  pm::g_epoch.fetch_add(1);
  return PM_OK;
}

pm_status pm_tables_info(uint64_t* attached_bytes, uint64_t* used_bytes, int32_t* tables) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PM_EDEVICE;
  std::lock_guard<std::mutex> lock(pm::g_mu);
  uint64_t a = 0, u = 0;
  int32_t t = 0;
  auto it = pm::g_dev.find(pm::pool_key(pm::kPoolCaller, dev));
  if (it != pm::g_dev.end()) {
    for (const pm::Region& r : it->second.regions) {
      a += r.bytes;
      u += r.used;
    }
    t = (int32_t)it->second.entries.size();
  }
  if (attached_bytes) *attached_bytes = a;
  if (used_bytes) *used_bytes = u;
  if (tables) *tables = t;
  return PM_OK;
}

}  // extern "C"
