// pm_tune.cpp -- the tuning table: launch-shape choices per (prime class,
// transform length, shape bucket), measured on the device by the tuning
// driver (paper_1905_04356_amd/tune.py) and stored as JSON next to libpm.so.
//
// The paper finds the thresholds between its multiplication variants
// experimentally, with separate values for small and large primes, because
// no variant wins everywhere (Section 2, "Polynomial matrix multiplication").
// Here every variant computes the same residues, so the table only picks the
// fastest launch shapes: column-pass stages, stages per LDS pass, block-step
// threads and tile, column item widths, register or LDS tile, MFMA or VALU
// pointwise, pipelined pointwise slots, and the batch and wrapped-length
// thresholds.
//
// Table format (JSON):
//   {"format": "pm-tune-1",
//    "global": {"wrap_min_log": 10, ...},
//    "entries": [{"prime_class": "direct_ge30", "log2_len": 13,
//                 "m_log2": 6, "n_log2": 6, "k_log2": 5,
//                 "knobs": {"blk_nt": 256, ...}, ...}, ...]}
// An entry matches a product when every selector it names equals the
// product's (prime_class: "direct_lt30", "direct_ge30" or "crt"; log2_len:
// log2 L; m_log2, n_log2, k_log2: ceil(log2) of m, n, k); the first match
// wins, and its knobs replace the defaults they name.  Other fields
// (measurements) are ignored.  The table is read on first use from
// $PM_TUNE_TABLE if set (empty: none), else tune_table.json beside
// libpm.so; a missing or invalid file leaves the defaults, which come from
// the PM_TUNE_* environment variables.  pm_tune_load installs a table at
// run time.
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pm.h"
#include "pm_plan.h"

namespace pm {

namespace {

int env_int(const char* name, int dflt, int lo, int hi) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  int x = atoi(v);
  return x < lo ? lo : x > hi ? hi : x;
}

Knobs env_knobs() {
  Knobs k;
  k.split = env_int("PM_TUNE_NTT_SPLIT", 4, 0, 5);
  k.maxr = env_int("PM_TUNE_NTT_MAXR", 4, 2, 4);
  k.blk_nt = env_int("PM_TUNE_NTT_BLK_NT", 256, 256, 512) > 256 ? 512 : 256;
  k.blk_tile_log = env_int("PM_TUNE_NTT_BLK_TILE_LOG", 13, 11, 15);
  k.colvec_fwd = env_int("PM_TUNE_NTT_COLVEC_FWD", 4, 1, 4);
  k.colvec_inv = env_int("PM_TUNE_NTT_COLVEC_INV", 4, 1, 4);
  k.reg_tile = env_int("PM_TUNE_NTT_REG_TILE", 1, 0, 1);
  k.pointwise = env_int("PM_TUNE_POINTWISE", 1, 0, 1);
  // up to 44 KiB of limb planes: 256 threads, so that several workgroups
  // share a CU; above, 512 threads wait for fewer load round trips each
  k.pw_small_lds = env_int("PM_TUNE_PW_SMALL_LDS", 44 * 1024, 0, 1 << 30);
  k.pw_pipe = env_int("PM_TUNE_PW_PIPE", -1, -1, 2);
  k.blk_nt_inv = 0;
  k.blk_tile_log_inv = 0;
  return k;
}

GlobalKnobs env_global() {
  GlobalKnobs g;
  g.lds_log = env_int("PM_TUNE_NTT_LDS_LOG", 14, 11, 15);
  g.split_min_log = env_int("PM_TUNE_NTT_SPLIT_MINLOG", 11, 2, 16);
  g.blk_pad = env_int("PM_TUNE_NTT_BLK_PAD", 0, 0, 64) & ~3;
  g.batch_tile_log = env_int("PM_TUNE_BATCH_TILE_LOG", 14, 11, 15);
  g.batch_pw_work = env_int("PM_TUNE_BATCH_PW_WORK", 8192, 1, 1 << 30);
  g.batch_pw_pipe_pts = env_int("PM_TUNE_BATCH_PW_PIPE_PTS", 16, 1, 1 << 20);
  g.batch_direct_max = env_int("PM_TUNE_BATCH_DIRECT_MAX", 2, 0, 1 << 20);
  g.batch_graph = env_int("PM_TUNE_BATCH_GRAPH", 1, 0, 1);
  {
    const char* e = getenv("PM_TUNE_WRAP");
    g.wrap_min_log = e && e[0] == '0' ? 99 : env_int("PM_TUNE_WRAP_MINLOG", 10, 1, 99);
  }
  g.wrap_top_div = 4;
  g.wrap_min_work_log = 25;
  g.vdm_max_d = env_int("PM_TUNE_VDM_MAXD", 64, 0, 1 << 20);
  g.min_wg = env_int("PM_TUNE_MIN_WG", 512, 0, 1 << 20);
  g.min_wg_unsplit = env_int("PM_TUNE_MIN_WG_UNSPLIT", 256, 0, 1 << 20);
  g.trunc34 = env_int("PM_TUNE_TRUNC34", 1, 0, 2);
  g.wrap_top_div_tr = 8;
  g.wrap_tr_max_log = 13;
  g.crt_fused = env_int("PM_TUNE_CRT_FUSED", 1, 0, 1);
  g.batch_single_min_log = env_int("PM_TUNE_BATCH_SINGLE_MIN_LOG", 25, 0, 62);
  g.col_fwd_mp = env_int("PM_TUNE_COL_FWD_MP", 1, 0, 1);
  g.lazy = env_int("PM_TUNE_LAZY", 1, 0, 1);
  return g;
}

struct Entry {
  int pclass = -1, logL = -1, m_log = -1, n_log = -1, k_log = -1;  // -1: any
  std::vector<std::pair<int, int>> set;  // (knob index, value)
};

struct Table {
  Knobs base;
  GlobalKnobs global;
  std::vector<Entry> entries;
  int source = 0;  // 0 defaults, 1 file, 2 caller text, -1 file unreadable
};

// ---- a small JSON reader (objects, arrays, strings, numbers, literals) -------

struct JVal {
  enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
  double num = 0;
  bool isint = false;
  long long inum = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
};

struct JParser {
  const char* p;
  const char* end;
  int depth = 0;
  bool ok = true;

  void ws() {
    while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
  }
  bool lit(const char* s) {
    const size_t n = strlen(s);
    if ((size_t)(end - p) < n || strncmp(p, s, n) != 0) return false;
    p += n;
    return true;
  }
  bool string(std::string* out) {
    if (p >= end || *p != '"') return false;
    ++p;
    while (p < end && *p != '"') {
      if (*p == '\\') {
        if (++p >= end) return false;
        switch (*p) {
          case '"': case '\\': case '/': out->push_back(*p); break;
          case 'n': out->push_back('\n'); break;
          case 't': out->push_back('\t'); break;
          default: return false;  // no other escapes in tuning tables
        }
        ++p;
      } else {
        out->push_back(*p++);
      }
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool number(JVal* v) {
    const char* s = p;
    if (p < end && (*p == '-' || *p == '+')) ++p;
    bool frac = false;
    while (p < end && ((*p >= '0' && *p <= '9') || *p == '.' || *p == 'e' || *p == 'E' ||
                       ((*p == '-' || *p == '+') && (p[-1] == 'e' || p[-1] == 'E')))) {
      if (*p == '.' || *p == 'e' || *p == 'E') frac = true;
      ++p;
    }
    if (p == s) return false;
    const std::string t(s, p);
    char* e = nullptr;
    v->kind = JVal::kNum;
    v->num = strtod(t.c_str(), &e);
    if (!e || *e) return false;
    v->isint = !frac;
    if (v->isint) v->inum = strtoll(t.c_str(), nullptr, 10);
    return true;
  }
  bool value(JVal* v) {
    if (++depth > 32) return false;
    ws();
    bool r = false;
    if (p >= end) {
      r = false;
    } else if (*p == '{') {
      ++p;
      v->kind = JVal::kObj;
      ws();
      if (p < end && *p == '}') {
        ++p;
        r = true;
      } else {
        for (;;) {
          ws();
          std::string key;
          if (!string(&key)) break;
          ws();
          if (p >= end || *p != ':') break;
          ++p;
          JVal x;
          if (!value(&x)) break;
          v->obj.emplace_back(key, std::move(x));
          ws();
          if (p < end && *p == ',') { ++p; continue; }
          if (p < end && *p == '}') { ++p; r = true; }
          break;
        }
      }
    } else if (*p == '[') {
      ++p;
      v->kind = JVal::kArr;
      ws();
      if (p < end && *p == ']') {
        ++p;
        r = true;
      } else {
        for (;;) {
          JVal x;
          if (!value(&x)) break;
          v->arr.push_back(std::move(x));
          ws();
          if (p < end && *p == ',') { ++p; continue; }
          if (p < end && *p == ']') { ++p; r = true; }
          break;
        }
      }
    } else if (*p == '"') {
      v->kind = JVal::kStr;
      r = string(&v->str);
    } else if (lit("true")) {
      v->kind = JVal::kBool; v->num = 1; r = true;
    } else if (lit("false")) {
      v->kind = JVal::kBool; r = true;
    } else if (lit("null")) {
      r = true;
    } else {
      r = number(v);
    }
    --depth;
    return r;
  }
};

// ---- knobs by name, with their admissible values ---------------------------

struct KnobDef {
  const char* name;
  int lo, hi;
};
const KnobDef kKnobs[] = {
    {"split", 0, 5},        {"maxr", 2, 4},        {"blk_nt", 256, 512},
    {"blk_tile_log", 11, 15}, {"colvec_fwd", 1, 4}, {"colvec_inv", 1, 4},
    {"reg_tile", 0, 1},     {"pointwise", 0, 1},   {"pw_small_lds", 0, 1 << 30},
    {"pw_pipe", -1, 2},     {"blk_nt_inv", 0, 512}, {"blk_tile_log_inv", 0, 15},
};
const KnobDef kGlobals[] = {
    {"lds_log", 11, 15},          {"split_min_log", 2, 16},    {"blk_pad", 0, 64},
    {"batch_tile_log", 11, 15},   {"batch_pw_work", 1, 1 << 30},
    {"batch_pw_pipe_pts", 1, 1 << 20}, {"batch_direct_max", 0, 1 << 20},
    {"batch_graph", 0, 1},        {"wrap_min_log", 1, 99},     {"wrap_top_div", 1, 1 << 20},
    {"wrap_min_work_log", 0, 62}, {"vdm_max_d", 0, 1 << 20}, {"min_wg", 0, 1 << 20},
    {"trunc34", 0, 2},            {"wrap_top_div_tr", 1, 1 << 20},
    {"wrap_tr_max_log", 0, 99},   {"crt_fused", 0, 1},
    {"batch_single_min_log", 0, 62}, {"col_fwd_mp", 0, 1},     {"lazy", 0, 1},
    {"min_wg_unsplit", 0, 1 << 20},
};

int* knob_slot(Knobs& k, int i) {
  int* f[] = {&k.split, &k.maxr, &k.blk_nt, &k.blk_tile_log, &k.colvec_fwd, &k.colvec_inv,
              &k.reg_tile, &k.pointwise, &k.pw_small_lds, &k.pw_pipe, &k.blk_nt_inv,
              &k.blk_tile_log_inv};
  return f[i];
}
int* global_slot(GlobalKnobs& g, int i) {
  int* f[] = {&g.lds_log, &g.split_min_log, &g.blk_pad, &g.batch_tile_log, &g.batch_pw_work,
              &g.batch_pw_pipe_pts, &g.batch_direct_max, &g.batch_graph, &g.wrap_min_log,
              &g.wrap_top_div, &g.wrap_min_work_log, &g.vdm_max_d, &g.min_wg, &g.trunc34,
              &g.wrap_top_div_tr, &g.wrap_tr_max_log, &g.crt_fused,
              &g.batch_single_min_log, &g.col_fwd_mp, &g.lazy, &g.min_wg_unsplit};
  return f[i];
}

bool valid_knob(int i, int v) {
  if (v < kKnobs[i].lo || v > kKnobs[i].hi) return false;
  const std::string n = kKnobs[i].name;
  if (n == "split") return v == 0 || v >= 2;
  if (n == "blk_nt") return v == 256 || v == 512;
  if (n == "blk_nt_inv") return v == 0 || v == 256 || v == 512;
  if (n == "blk_tile_log_inv") return v == 0 || v >= 11;
  if (n == "colvec_fwd" || n == "colvec_inv") return v == 1 || v == 2 || v == 4;
  return true;
}

bool int_of(const JVal& v, int* out) {
  if (v.kind != JVal::kNum || !v.isint || v.inum < -(1ll << 31) || v.inum >= (1ll << 31))
    return false;
  *out = (int)v.inum;
  return true;
}

// Parse a table; false (and *why) on any error.
bool parse_table(const char* text, size_t len, Table* T, std::string* why) {
  JParser P{text, text + len};
  JVal root;
  if (!P.value(&root)) { *why = "not JSON"; return false; }
  P.ws();
  if (P.p != P.end) { *why = "trailing characters"; return false; }
  if (root.kind != JVal::kObj) { *why = "top level is not an object"; return false; }
  for (auto& kv : root.obj) {
    if (kv.first == "format") {
      if (kv.second.kind != JVal::kStr || kv.second.str != "pm-tune-1") {
        *why = "format is not pm-tune-1";
        return false;
      }
    } else if (kv.first == "global") {
      if (kv.second.kind != JVal::kObj) { *why = "global is not an object"; return false; }
      for (auto& g : kv.second.obj) {
        int idx = -1;
        for (int i = 0; i < (int)(sizeof kGlobals / sizeof kGlobals[0]); ++i)
          if (g.first == kGlobals[i].name) idx = i;
        int v;
        if (idx < 0 || !int_of(g.second, &v) || v < kGlobals[idx].lo || v > kGlobals[idx].hi) {
          *why = "bad global knob " + g.first;
          return false;
        }
        *global_slot(T->global, idx) = idx == 2 ? v & ~3 : v;
      }
    } else if (kv.first == "entries") {
      if (kv.second.kind != JVal::kArr) { *why = "entries is not an array"; return false; }
      for (auto& e : kv.second.arr) {
        if (e.kind != JVal::kObj) { *why = "entry is not an object"; return false; }
        Entry E;
        for (auto& f : e.obj) {
          int v;
          if (f.first == "prime_class") {
            const std::string& c = f.second.str;
            if (f.second.kind != JVal::kStr) { *why = "bad prime_class"; return false; }
            E.pclass = c == "direct_lt30" ? kClassDirectLt30
                       : c == "direct_ge30" ? kClassDirectGe30
                       : c == "crt" ? kClassCrt : -2;
            if (E.pclass == -2) { *why = "bad prime_class " + c; return false; }
          } else if (f.first == "log2_len" || f.first == "m_log2" || f.first == "n_log2" ||
                     f.first == "k_log2") {
            if (!int_of(f.second, &v) || v < 0 || v > 30) {
              *why = "bad selector " + f.first;
              return false;
            }
            (f.first == "log2_len" ? E.logL
             : f.first == "m_log2" ? E.m_log
             : f.first == "n_log2" ? E.n_log : E.k_log) = v;
          } else if (f.first == "knobs") {
            if (f.second.kind != JVal::kObj) { *why = "knobs is not an object"; return false; }
            for (auto& kb : f.second.obj) {
              int idx = -1;
              for (int i = 0; i < (int)(sizeof kKnobs / sizeof kKnobs[0]); ++i)
                if (kb.first == kKnobs[i].name) idx = i;
              if (idx < 0 || !int_of(kb.second, &v) || !valid_knob(idx, v)) {
                *why = "bad knob " + kb.first;
                return false;
              }
              E.set.emplace_back(idx, v);
            }
          }  // other fields: measurements, ignored
        }
        T->entries.push_back(std::move(E));
      }
    }  // other top-level fields: ignored
  }
  return true;
}

std::mutex g_mu;
std::shared_ptr<const Table> g_table;
std::atomic<uint64_t> g_epoch{0};
bool g_loaded = false;

std::shared_ptr<Table> fresh_table(int source) {
  auto t = std::make_shared<Table>();
  t->base = env_knobs();
  t->global = env_global();
  t->source = source;
  return t;
}

void install(std::shared_ptr<const Table> t) {
  g_table = std::move(t);
  g_epoch.fetch_add(1);
}

std::string default_path() {
  const char* e = getenv("PM_TUNE_TABLE");
  if (e) return e;  // empty: no table
  Dl_info info;
  if (!dladdr((const void*)&tune_epoch, &info) || !info.dli_fname) return "";
  std::string so = info.dli_fname;
  const size_t slash = so.rfind('/');
  return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) +
         "/tune_table.json";
}

// The table from the default file (or the defaults alone).
std::shared_ptr<const Table> load_default() {
  const std::string path = default_path();
  if (path.empty()) return fresh_table(0);
  FILE* f = fopen(path.c_str(), "rb");
  if (!f) return fresh_table(0);
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  fclose(f);
  auto t = fresh_table(1);
  std::string why;
  if (!parse_table(text.data(), text.size(), t.get(), &why)) {
    fprintf(stderr, "libpm: ignoring tuning table %s (%s)\n", path.c_str(), why.c_str());
    return fresh_table(-1);
  }
  return t;
}

std::shared_ptr<const Table> current() {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_loaded) {
    install(load_default());
    g_loaded = true;
  }
  return g_table;
}

int ceil_log2_int(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

}  // namespace

uint64_t tune_epoch() { return g_epoch.load(); }

Knobs tuned_knobs(int pclass, int logL, int m, int n, int k, int* entry) {
  alloc_point();  // the table snapshot
  const std::shared_ptr<const Table> t = current();
  Knobs kn = t->base;
  if (entry) *entry = -1;
  const int ml = ceil_log2_int(m), nl = ceil_log2_int(n), kl = ceil_log2_int(k);
  for (size_t i = 0; i < t->entries.size(); ++i) {
    const Entry& E = t->entries[i];
    if ((E.pclass >= 0 && E.pclass != pclass) || (E.logL >= 0 && E.logL != logL) ||
        (E.m_log >= 0 && E.m_log != ml) || (E.n_log >= 0 && E.n_log != nl) ||
        (E.k_log >= 0 && E.k_log != kl))
      continue;
    for (auto& kv : E.set) *knob_slot(kn, kv.first) = kv.second;
    if (entry) *entry = (int)i;
    break;
  }
  return kn;
}

GlobalKnobs global_knobs() { return current()->global; }

Knobs base_knobs() { return current()->base; }

}  // namespace pm

extern "C" {

pm_status pm_tune_load(const char* json) {
  return (pm_status)pm::guarded([&] {
    pm::alloc_point();
    std::shared_ptr<const pm::Table> t;
    if (!json) {
      t = pm::load_default();
    } else {
      auto n = pm::fresh_table(2);
      std::string why;
      if (*json && !pm::parse_table(json, strlen(json), n.get(), &why)) return (int)PM_EINVAL;
      if (!*json) n->source = 0;
      t = n;
    }
    std::lock_guard<std::mutex> lock(pm::g_mu);
    pm::install(t);
    pm::g_loaded = true;
    return (int)PM_OK;
  });
}

pm_status pm_tune_info(int32_t* entries, int32_t* source) {
  return (pm_status)pm::guarded([&] {
    const std::shared_ptr<const pm::Table> t = pm::current();
    if (entries) *entries = (int32_t)t->entries.size();
    if (source) *source = t->source;
    return (int)PM_OK;
  });
}

}  // extern "C"
