// tune.hip -- autotuner of the launch shapes and work splits (rst_option), with
// a per-context cache that can be written to and read from a JSON file.
//
// The search is coordinate descent from the context's current setting: for
// each knob of the method, every candidate value is timed (median of `reps`
// runs of the whole call, HIP events on the context stream, after one warm-up
// run) and its output is checked on the device against component labels
// computed once before the search; a candidate whose output fails, or whose
// calls return another status than the starting setting's, is rejected.  The best value is kept before the next knob.
// Entries are keyed by (GPU architecture, method, floor(log2 n),
// floor(log2 average degree)) so that one tuning serves graphs of a similar
// size and density.
#include "rst_internal.h"

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace rst {

struct TuneEntry {
  float ms = 0.f;
  std::map<int, int64_t> values;   // rst_option -> value
};

struct TuneCache {
  std::map<std::string, TuneEntry> entries;
};

void tune_free(rst_ctx *ctx) {
  delete ctx->tune;
  ctx->tune = nullptr;
}

static std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

static int floor_log2(double x) { return x < 1.0 ? 0 : (int)std::floor(std::log2(x)); }

static std::string tune_key(const rst_ctx *ctx, const rst_csr *g, rst_method method) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "%s:%s:n%d:d%d", arch_name(ctx->device).c_str(),
                method == RST_BFS ? "bfs" : "gconn", floor_log2((double)g->n),
                floor_log2((double)g->nnz / (double)g->n));
  return buf;
}

struct Knob {
  rst_option opt;
  std::vector<int64_t> values;
};

static std::vector<Knob> knobs_for(rst_method method) {
  if (method == RST_BFS)
    return {{RST_OPT_BFS_LEVELS_PER_SYNC, {4, 8, 16, 32, 64, 128}},
            {RST_OPT_BFS_GRID, {0, 512, 1024, 2048, 4096}},
            {RST_OPT_BFS_HEAVY_DEGREE, {256, 1024, 4096, 16384}}};
  // hooking variant and its sampling first: they decide which kernels run
  return {{RST_OPT_HOOK_MODE, {1, 2}},
          {RST_OPT_HOOK_SAMPLE, {-1, 0, 1, 2, 3}},
          {RST_OPT_SWEEP_BLOCK, {64, 128, 256, 512, 1024}},
          {RST_OPT_HEAVY_DEGREE, {256, 1024, 4096, 16384}},
          {RST_OPT_RANK_ELEMS_PER_THREAD, {1, 2, 4, 8}},
          {RST_OPT_RANK_STRIDE, {0, 4, 8, 16, 32, 64}}};
}

// Device check of a candidate's output against component labels computed
// once, before the search, under the settings the search started from: a
// knob-dependent fault in the library's own hooking cannot make the labels
// and the parent array wrong in the same way.  *bad = failed checks.
static rst_status verify_against(rst_ctx *ctx, const rst_csr *g, int32_t root,
                                 const int32_t *ref_label, const int32_t *parent, int64_t *bad) {
  const int64_t n = g->n;
  RST_TRY(ws_reserve(ctx, ws_bytes(64, 4) + 2 * ws_bytes(n, 4)));
  int32_t *vc = ws_take<int32_t>(ctx, 64);
  int32_t *anc0 = ws_take<int32_t>(ctx, n);
  int32_t *anc1 = ws_take<int32_t>(ctx, n);
  RST_TRY(enqueue_fill(ctx, vc, 1, 0));
  RST_TRY(enqueue_fill(ctx, vc + 1, 1, 0x7fffffff));
  RST_TRY(enqueue_verify(ctx, g, root, ref_label, parent, anc0, anc1, vc));
  RST_HIP(hipMemcpyAsync(ctx->host_pinned + 40, vc, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                         ctx->stream));
  RST_HIP(hipStreamSynchronize(ctx->stream));
  *bad = ctx->host_pinned[40];
  return RST_OK;
}

// Median time of `reps` calls (after one warm-up call); *ok = every call
// returned `want` (the status of the starting setting) and the last output
// passes the check against the reference labels.
static rst_status time_config(rst_ctx *ctx, const rst_csr *g, int32_t root, rst_method method,
                              int32_t reps, int32_t *parent, const int32_t *ref_label,
                              rst_status want, hipEvent_t e0, hipEvent_t e1, float *ms, bool *ok) {
  bool same = true;
  rst_status s = rst_spanning_tree(ctx, g, root, method, parent, nullptr);
  if (s != RST_OK && s != RST_E_DISCONNECTED) return s;
  same = same && s == want;
  std::vector<float> t;
  for (int r = 0; r < reps; ++r) {
    RST_HIP(hipEventRecord(e0, ctx->stream));
    s = rst_spanning_tree(ctx, g, root, method, parent, nullptr);
    if (s != RST_OK && s != RST_E_DISCONNECTED) return s;
    same = same && s == want;
    RST_HIP(hipEventRecord(e1, ctx->stream));
    RST_HIP(hipEventSynchronize(e1));
    float x = 0.f;
    RST_HIP(hipEventElapsedTime(&x, e0, e1));
    t.push_back(x);
  }
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  int64_t bad = 0;
  RST_TRY(verify_against(ctx, g, root, ref_label, parent, &bad));
  *ok = same && bad == 0;
  return RST_OK;
}

// ---------------------------------------------------------------------------
// cache file: {"format": "rst-tune-1", "entries": {"<key>": {"ms": <float>,
// "options": {"<option id>": <int>, ...}}, ...}}
// ---------------------------------------------------------------------------

struct Reader {
  const std::string &s;
  size_t i = 0;
  explicit Reader(const std::string &t) : s(t) {}
  void ws() { while (i < s.size() && std::isspace((unsigned char)s[i])) ++i; }
  bool eat(char c) { ws(); if (i < s.size() && s[i] == c) { ++i; return true; } return false; }
  bool str(std::string *out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    size_t j = s.find('"', i + 1);
    if (j == std::string::npos) return false;
    *out = s.substr(i + 1, j - i - 1);
    i = j + 1;
    return true;
  }
  bool num(double *out) {
    ws();
    const char *b = s.c_str() + i;
    char *e = nullptr;
    *out = std::strtod(b, &e);
    if (e == b) return false;
    i += (size_t)(e - b);
    return true;
  }
};

static bool parse_entry(Reader &r, TuneEntry *e) {
  if (!r.eat('{')) return false;
  if (r.eat('}')) return true;
  do {
    std::string k;
    if (!r.str(&k) || !r.eat(':')) return false;
    if (k == "ms") {
      double x;
      if (!r.num(&x)) return false;
      e->ms = (float)x;
    } else if (k == "options") {
      if (!r.eat('{')) return false;
      if (!r.eat('}')) {
        do {
          std::string ok;
          double x;
          if (!r.str(&ok) || !r.eat(':') || !r.num(&x)) return false;
          e->values[std::atoi(ok.c_str())] = (int64_t)x;
        } while (r.eat(','));
        if (!r.eat('}')) return false;
      }
    } else {
      return false;
    }
  } while (r.eat(','));
  return r.eat('}');
}

static bool parse_cache(const std::string &text, TuneCache *c) {
  Reader r(text);
  if (!r.eat('{')) return false;
  bool have_format = false;
  do {
    std::string k;
    if (!r.str(&k) || !r.eat(':')) return false;
    if (k == "format") {
      std::string f;
      if (!r.str(&f) || f != "rst-tune-1") return false;
      have_format = true;
    } else if (k == "entries") {
      if (!r.eat('{')) return false;
      if (!r.eat('}')) {
        do {
          std::string key;
          TuneEntry e;
          if (!r.str(&key) || !r.eat(':') || !parse_entry(r, &e)) return false;
          c->entries[key] = e;
        } while (r.eat(','));
        if (!r.eat('}')) return false;
      }
    } else {
      return false;
    }
  } while (r.eat(','));
  return r.eat('}') && have_format;
}

}  // namespace rst

using namespace rst;

extern "C" {

rst_status rst_autotune(rst_ctx *ctx, const rst_csr *g, int32_t root, rst_method method,
                        int32_t reps, rst_tune_result *result) {
  if (!ctx || !g || reps < 1 || reps > 101) return RST_E_INVAL;
  if (method == RST_AUTO) method = RST_GCONN_EULER;
  if (method != RST_GCONN_EULER && method != RST_BFS) return RST_E_INVAL;
  if (g->n < 1 || root < 0 || root >= g->n) return RST_E_INVAL;
  RST_HIP(hipSetDevice(ctx->device));
  // the output buffer and the reference labels (component minima, computed
  // once under the starting settings)
  int32_t *parent = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&parent), 2 * (size_t)g->n * sizeof(int32_t)) !=
      hipSuccess) {
    (void)hipGetLastError();
    return RST_E_NOMEM;
  }
  int32_t *ref_label = parent + g->n;
  int64_t ref_comps = 0;
  {
    const rst_status ls = rst_components(ctx, g, ref_label, &ref_comps);
    if (ls != RST_OK) { (void)hipFree(parent); return ls; }
  }
  const rst_status want = ref_comps > 1 ? RST_E_DISCONNECTED : RST_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rst_status status = RST_OK;
  float ms_default = 0.f, ms_best = 0.f;
  int candidates = 0, rejected = 0;
  const std::vector<Knob> knobs = knobs_for(method);
  do {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      status = RST_E_DEVICE;
      break;
    }
    bool ok = false;
    status = time_config(ctx, g, root, method, reps, parent, ref_label, want, e0, e1, &ms_default,
                         &ok);
    if (status != RST_OK) break;
    if (!ok) { status = RST_E_DEVICE; break; }   // the current setting itself fails
    ms_best = ms_default;
    for (const Knob &k : knobs) {
      int64_t best_v = 0;
      (void)rst_get_option(ctx, k.opt, &best_v);
      for (int64_t v : k.values) {
        if (v == best_v) continue;
        if (rst_set_option(ctx, k.opt, v) != RST_OK) continue;
        float ms = 0.f;
        status = time_config(ctx, g, root, method, reps, parent, ref_label, want, e0, e1, &ms,
                             &ok);
        if (status != RST_OK) break;
        ++candidates;
        if (!ok) { ++rejected; continue; }
        if (ms < ms_best) { ms_best = ms; best_v = v; }
      }
      (void)rst_set_option(ctx, k.opt, best_v);
      if (status != RST_OK) break;
    }
  } while (false);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(parent);
  if (status != RST_OK) return status;

  if (!ctx->tune) ctx->tune = new TuneCache;
  TuneEntry &e = ctx->tune->entries[tune_key(ctx, g, method)];
  e.ms = ms_best;
  e.values.clear();
  for (const Knob &k : knobs) {
    int64_t v = 0;
    (void)rst_get_option(ctx, k.opt, &v);
    e.values[(int)k.opt] = v;
  }
  if (result) {
    std::memset(result, 0, sizeof(*result));
    int i = 0;
    for (const auto &kv : e.values) {
      if (i >= 8) break;
      result->options[i] = kv.first;
      result->values[i] = kv.second;
      ++i;
    }
    result->num_options = i;
    result->ms_best = ms_best;
    result->ms_default = ms_default;
    result->candidates = candidates;
    result->rejected = rejected;
  }
  return RST_OK;
}

rst_status rst_tune_save(const rst_ctx *ctx, const char *path) {
  if (!ctx || !path) return RST_E_INVAL;
  FILE *f = std::fopen(path, "w");
  if (!f) return RST_E_INVAL;
  std::fprintf(f, "{\"format\": \"rst-tune-1\", \"entries\": {");
  bool first = true;
  if (ctx->tune) {
    for (const auto &kv : ctx->tune->entries) {
      std::fprintf(f, "%s\n  \"%s\": {\"ms\": %.6g, \"options\": {", first ? "" : ",",
                   kv.first.c_str(), (double)kv.second.ms);
      bool f2 = true;
      for (const auto &ov : kv.second.values) {
        std::fprintf(f, "%s\"%d\": %lld", f2 ? "" : ", ", ov.first, (long long)ov.second);
        f2 = false;
      }
      std::fprintf(f, "}}");
      first = false;
    }
  }
  std::fprintf(f, "\n}}\n");
  const bool ok = std::ferror(f) == 0;
  return (std::fclose(f) == 0 && ok) ? RST_OK : RST_E_INVAL;
}

rst_status rst_tune_load(rst_ctx *ctx, const char *path, const rst_csr *g, rst_method method,
                         int32_t *applied) {
  if (!ctx || !path) return RST_E_INVAL;
  if (applied) *applied = 0;
  FILE *f = std::fopen(path, "r");
  if (!f) return RST_E_INVAL;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
  std::fclose(f);
  TuneCache c;
  if (!parse_cache(text, &c)) return RST_E_INVAL;
  // every value is checked by rst_set_option on a scratch context before
  // anything is merged or applied
  rst_ctx probe;
  for (const auto &kv : c.entries)
    for (const auto &ov : kv.second.values)
      if (ov.first < 0 || ov.first >= RST_NUM_OPTIONS || ov.first == RST_OPT_VALIDATE ||
          rst_set_option(&probe, (rst_option)ov.first, ov.second) != RST_OK)
        return RST_E_INVAL;
  if (!ctx->tune) ctx->tune = new TuneCache;
  for (const auto &kv : c.entries) ctx->tune->entries[kv.first] = kv.second;
  if (!g) return RST_OK;
  if (method == RST_AUTO) method = RST_GCONN_EULER;
  const auto it = ctx->tune->entries.find(tune_key(ctx, g, method));
  if (it == ctx->tune->entries.end()) return RST_OK;
  for (const auto &ov : it->second.values) (void)rst_set_option(ctx, (rst_option)ov.first, ov.second);
  if (applied) *applied = 1;
  return RST_OK;
}

}  // extern "C"
