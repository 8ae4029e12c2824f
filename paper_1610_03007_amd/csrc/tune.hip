// Tuning cache and search. A table of tuning entries keyed by (GPU
// architecture, build mode, log2 of the input size, bits per character code)
// chooses the radix-sort tile shape, the persistent sweep grid, the lazy-ISA
// threshold and the round-0 key width for builds that have no explicit tuning.
// The table is read from and written to a small JSON file; sa_tune fills it by
// timing candidate tunings on a caller's input. No choice here changes a
// result, only the time a build takes.

#include <cctype>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>

#include "driver.h"

namespace drv {

// ---------------------------------------------------------------------------
// A small JSON reader: objects, arrays, strings (no escapes beyond \" \\ \/),
// numbers, true/false/null. Enough for the cache files written below.

namespace {

struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  double num = 0;
  bool b = false;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* k) const {
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* p;
  const char* end;
  int depth = 0;
  void ws() {
    while (p < end && std::isspace(static_cast<unsigned char>(*p))) ++p;
  }
  bool lit(const char* s) {
    const size_t k = std::strlen(s);
    if (size_t(end - p) < k || std::strncmp(p, s, k) != 0) return false;
    p += k;
    return true;
  }
  bool string(std::string& out) {
    if (p >= end || *p != '"') return false;
    ++p;
    out.clear();
    while (p < end && *p != '"') {
      char ch = *p++;
      if (ch == '\\') {
        if (p >= end) return false;
        ch = *p++;
        if (ch != '"' && ch != '\\' && ch != '/') return false;
      }
      out.push_back(ch);
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool value(JVal& v) {
    if (++depth > 32) return false;
    ws();
    if (p >= end) return false;
    bool ok = true;
    if (*p == '{') {
      ++p;
      v.kind = JVal::OBJ;
      ws();
      if (p < end && *p == '}') {
        ++p;
      } else {
        for (;;) {
          ws();
          std::string k;
          JVal x;
          if (!string(k)) return false;
          ws();
          if (p >= end || *p != ':') return false;
          ++p;
          if (!value(x)) return false;
          v.obj.emplace_back(std::move(k), std::move(x));
          ws();
          if (p < end && *p == ',') {
            ++p;
            continue;
          }
          if (p < end && *p == '}') {
            ++p;
            break;
          }
          return false;
        }
      }
    } else if (*p == '[') {
      ++p;
      v.kind = JVal::ARR;
      ws();
      if (p < end && *p == ']') {
        ++p;
      } else {
        for (;;) {
          JVal x;
          if (!value(x)) return false;
          v.arr.push_back(std::move(x));
          ws();
          if (p < end && *p == ',') {
            ++p;
            continue;
          }
          if (p < end && *p == ']') {
            ++p;
            break;
          }
          return false;
        }
      }
    } else if (*p == '"') {
      v.kind = JVal::STR;
      ok = string(v.str);
    } else if (lit("true")) {
      v.kind = JVal::BOOL;
      v.b = true;
    } else if (lit("false")) {
      v.kind = JVal::BOOL;
    } else if (lit("null")) {
      v.kind = JVal::NUL;
    } else {
      const std::string s(p, size_t(std::min<ptrdiff_t>(end - p, 64)));
      char* e = nullptr;
      v.num = std::strtod(s.c_str(), &e);
      if (e == s.c_str()) return false;
      v.kind = JVal::NUM;
      p += e - s.c_str();
    }
    --depth;
    return ok;
  }
};

bool num_field(const JVal& o, const char* k, double lo, double hi, double* out) {
  const JVal* v = o.get(k);
  if (!v || v->kind != JVal::NUM || !(v->num >= lo && v->num <= hi)) return false;
  *out = v->num;
  return true;
}

}  // namespace

// Checks the knobs the way sa_ctx_set_tuning does.
bool tuning_valid(const sa_tuning& t) {
  const u32 rb = t.radix_bits ? t.radix_bits : u32(kRadixBits);
  if (rb < u32(kRadixBitsMin) || rb > u32(kRadixBitsMax)) return false;
  if (t.sort_match > 1) return false;
  const int block = t.sort_block ? int(t.sort_block) : 256;
  if (!onesweep_supported(int(t.sort_items), block, t.sort_match == 1, int(rb))) return false;
  if (t.lazy_ratio < 3 || t.round0_full > 1 || t.sort_wgs_per_cu > 16) return false;
  if (t.rounds_ahead > 64 || t.round_graphs > 1) return false;
  if (t.prefix_mult != 0 && t.prefix_mult != 2 && t.prefix_mult != 4) return false;
  if (t.isa_direct > 1) return false;
  return true;
}

sa_tuning default_tuning() {
  sa_tuning t;
  std::memset(&t, 0, sizeof(t));
  t.sort_items = kSortItemsDefault;
  t.sort_block = kSortBlockDefault;
  t.lazy_ratio = u32(kLazyRatioDefault);
  t.round0_full = 0;
  t.sort_wgs_per_cu = 0;
  t.radix_bits = u32(kRadixBits);
  t.prefix_mult = 2;
  return t;
}

sa_status tune_parse(const std::string& text, TuneTable& out) {
  out.entries.clear();
  JParser jp{text.data(), text.data() + text.size()};
  JVal root;
  if (!jp.value(root)) return SA_EINVAL;
  jp.ws();
  if (jp.p != jp.end || root.kind != JVal::OBJ) return SA_EINVAL;
  const JVal* fmt = root.get("format");
  if (!fmt || fmt->kind != JVal::STR || fmt->str != kTuneFormat) return SA_EINVAL;
  const JVal* ents = root.get("entries");
  if (!ents || ents->kind != JVal::ARR) return SA_EINVAL;
  for (const JVal& e : ents->arr) {
    if (e.kind != JVal::OBJ) return SA_EINVAL;
    TuneEntry te;
    const JVal* arch = e.get("arch");
    const JVal* mode = e.get("mode");
    if (!arch || arch->kind != JVal::STR || !mode || mode->kind != JVal::STR) return SA_EINVAL;
    if (mode->str != "single" && mode->str != "batch") return SA_EINVAL;
    te.arch = arch->str;
    te.mode = mode->str;
    double v;
    te.t = default_tuning();
    if (!num_field(e, "log2n", 0, 63, &v)) return SA_EINVAL;
    te.log2n = u32(v);
    if (!num_field(e, "code_bits", 0, 9, &v)) return SA_EINVAL;
    te.code_bits = u32(v);
    if (!num_field(e, "sort_items", 0, 64, &v)) return SA_EINVAL;
    te.t.sort_items = u32(v);
    if (!num_field(e, "sort_wgs_per_cu", 0, 16, &v)) return SA_EINVAL;
    te.t.sort_wgs_per_cu = u32(v);
    te.t.sort_block = kSortBlock;  // entries without the field predate 512-thread sweeps
    if (e.get("sort_block")) {
      if (!num_field(e, "sort_block", 0, 512, &v)) return SA_EINVAL;
      te.t.sort_block = u32(v);
    }
    if (!num_field(e, "lazy_ratio", 3, 1e9, &v)) return SA_EINVAL;
    te.t.lazy_ratio = u32(v);
    if (!num_field(e, "round0_full", 0, 1, &v)) return SA_EINVAL;
    te.t.round0_full = u32(v);
    te.t.sort_match = 0;  // entries without the field predate the match choice
    if (e.get("sort_match")) {
      if (!num_field(e, "sort_match", 0, 1, &v)) return SA_EINVAL;
      te.t.sort_match = u32(v);
    }
    te.t.radix_bits = u32(kRadixBits);  // entries without the field predate the width choice
    if (e.get("radix_bits")) {
      if (!num_field(e, "radix_bits", kRadixBitsMin, kRadixBitsMax, &v)) return SA_EINVAL;
      te.t.radix_bits = u32(v);
    }
    te.t.prefix_mult = 2;  // entries without the field predate quadrupling
    if (e.get("prefix_mult")) {
      if (!num_field(e, "prefix_mult", 2, 4, &v)) return SA_EINVAL;
      te.t.prefix_mult = u32(v);
    }
    if (!tuning_valid(te.t)) return SA_EINVAL;
    te.ms = num_field(e, "ms", 0, 1e12, &v) ? v : 0.0;
    out.entries.push_back(te);
  }
  return SA_OK;
}

sa_status tune_load(const char* path, TuneTable& out) {
  out.entries.clear();
  std::ifstream f(path, std::ios::binary);
  if (!f) return SA_OK;  // no cache yet: an empty table
  std::stringstream ss;
  ss << f.rdbuf();
  if (ss.str().size() > (size_t(1) << 24)) return SA_EINVAL;
  return tune_parse(ss.str(), out);
}

std::string tune_format(const TuneTable& t) {
  std::ostringstream o;
  o << "{\n  \"format\": \"" << kTuneFormat << "\",\n  \"entries\": [";
  for (size_t k = 0; k < t.entries.size(); ++k) {
    const TuneEntry& e = t.entries[k];
    char ms[64];
    std::snprintf(ms, sizeof(ms), "%.4f", e.ms);
    o << (k ? ",\n" : "\n") << "    {\"arch\": \"" << e.arch << "\", \"mode\": \"" << e.mode
      << "\", \"log2n\": " << e.log2n << ", \"code_bits\": " << e.code_bits
      << ", \"sort_items\": " << e.t.sort_items << ", \"sort_wgs_per_cu\": "
      << e.t.sort_wgs_per_cu << ", \"sort_block\": " << e.t.sort_block
      << ", \"sort_match\": " << e.t.sort_match
      << ", \"radix_bits\": " << (e.t.radix_bits ? e.t.radix_bits : u32(kRadixBits))
      << ", \"prefix_mult\": " << (e.t.prefix_mult == 4 ? 4u : 2u)
      << ", \"lazy_ratio\": " << e.t.lazy_ratio
      << ", \"round0_full\": " << e.t.round0_full << ", \"ms\": " << ms << "}";
  }
  o << "\n  ]\n}\n";
  return o.str();
}

sa_status tune_save(const char* path, const TuneTable& t) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) return SA_EINVAL;
    f << tune_format(t);
    if (!f) return SA_EINVAL;
  }
  if (std::rename(tmp.c_str(), path) != 0) return SA_EINVAL;
  return SA_OK;
}

// The entry for a build: same architecture and mode, the nearest size bucket
// within two binary orders of magnitude, then the nearest code width (0 on
// either side matches any width). Null when nothing is close enough.
const TuneEntry* tune_lookup(const TuneTable& t, const std::string& arch, const char* mode,
                             u32 log2n, u32 code_bits) {
  const TuneEntry* best = nullptr;
  long best_score = 0;
  for (const TuneEntry& e : t.entries) {
    if (e.arch != arch || e.mode != mode) continue;
    const long dn = std::labs(long(e.log2n) - long(log2n));
    if (dn > 2) continue;
    const long dc = (e.code_bits == 0 || code_bits == 0)
                        ? 0
                        : std::labs(long(e.code_bits) - long(code_bits));
    const long score = dn * 16 + dc;
    if (!best || score < best_score) {
      best = &e;
      best_score = score;
    }
  }
  return best;
}

void tune_upsert(TuneTable& t, const TuneEntry& e) {
  for (TuneEntry& x : t.entries) {
    if (x.arch == e.arch && x.mode == e.mode && x.log2n == e.log2n &&
        x.code_bits == e.code_bits) {
      x = e;
      return;
    }
  }
  t.entries.push_back(e);
}

void apply_tuning(sa_ctx* c, const sa_tuning& t) {
  c->sort_items = int(t.sort_items);
  c->sort_block = t.sort_block ? int(t.sort_block) : kSortBlock;
  c->lazy_ratio = t.lazy_ratio;
  c->round0_trim = t.round0_full ? 0 : 1;
  c->sort_wgs_per_cu = int(t.sort_wgs_per_cu);
  c->sort_match = int(t.sort_match);
  c->rounds_ahead = t.rounds_ahead;
  c->graphs = t.round_graphs == 0;
  c->radix_bits = t.radix_bits ? int(t.radix_bits) : kRadixBits;
  c->prefix_mult = t.prefix_mult == 4 ? 4 : 2;
  c->stage_isa = t.isa_direct == 0;
}

sa_tuning current_tuning(const sa_ctx* c) {
  sa_tuning t;
  std::memset(&t, 0, sizeof(t));
  t.sort_items = u32(c->sort_items);
  t.sort_block = u32(c->sort_block);
  t.lazy_ratio = u32(c->lazy_ratio);
  t.round0_full = c->round0_trim ? 0u : 1u;
  t.sort_wgs_per_cu = u32(c->sort_wgs_per_cu);
  t.sort_match = u32(c->sort_match);
  t.radix_bits = u32(c->radix_bits);
  t.rounds_ahead = c->rounds_ahead;
  t.round_graphs = c->graphs ? 0u : 1u;
  t.prefix_mult = u32(c->prefix_mult);
  t.isa_direct = c->stage_isa ? 0u : 1u;
  return t;
}

u32 log2_floor(u64 n) { return n ? u32(63 - __builtin_clzll(n)) : 0; }

// Chooses the knobs of the next build: the explicit tuning if the caller set
// one, else the cache entry for this input, else the defaults.
void resolve_tuning(sa_ctx* c, const char* mode, u64 n, u32 code_bits) {
  c->tuned_from_cache = 0;
  if (c->tuning_explicit) {
    apply_tuning(c, c->explicit_tuning);
    return;
  }
  const TuneEntry* e =
      c->tune ? tune_lookup(*c->tune, c->arch, mode, log2_floor(n), code_bits) : nullptr;
  if (e) {
    apply_tuning(c, e->t);
    c->tuned_from_cache = 1;
  } else {
    apply_tuning(c, default_tuning());
  }
}

}  // namespace drv

using namespace drv;

namespace {

// Times one build with the context's current knobs: the best of `reps` runs
// after one warm-up, in milliseconds on the stream's clock.
sa_status time_build(sa_ctx* c, const u8* text, const u64* off, u32 T, u32* d_sa, hipStream_t s,
                     u32 reps, double* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return SA_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SA_EDEVICE;
  }
  sa_status st = SA_OK;
  double best = 0;
  for (u32 r = 0; r <= reps && st == SA_OK; ++r) {
    if (hipEventRecord(e0, s) != hipSuccess) {
      st = SA_EDEVICE;
      break;
    }
    st = T == 1 ? build_rounds(c, text, off[1], 0, d_sa, nullptr, s)
                : build_batch_impl(c, text, off, T, d_sa, s);
    if (st != SA_OK) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = SA_EDEVICE;
      break;
    }
    float t = 0;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      st = SA_EDEVICE;
      break;
    }
    if (r > 0 && (best == 0 || t < best)) best = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return st;
}

}  // namespace

extern "C" {

sa_status sa_tune(sa_ctx* ctx, const uint8_t* d_texts, const uint64_t* h_offsets,
                  uint32_t num_texts, uint32_t* d_sas, void* stream, uint32_t reps,
                  sa_tuning* best_out, double* best_ms) {
  if (!ctx || !h_offsets || num_texts == 0 || !d_texts || !d_sas) return SA_EINVAL;
  if (reps == 0) reps = 3;
  if (reps > 100) return SA_EINVAL;
  if (h_offsets[0] != 0) return SA_EINVAL;
  for (u32 t = 0; t < num_texts; ++t)
    if (h_offsets[t + 1] < h_offsets[t]) return SA_EINVAL;
  const u64 N = h_offsets[num_texts];
  if (N == 0) return SA_EINVAL;
  if (!ctx->tune) {
    ctx->tune = new (std::nothrow) TuneTable();
    if (!ctx->tune) return SA_ENOMEM;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // The search sets the knobs directly; the caller's explicit tuning and the
  // statistics are put back afterwards.
  const bool was_explicit = ctx->tuning_explicit;
  const bool was_trace = ctx->trace;
  ctx->tuning_explicit = true;
  ctx->trace = false;
  sa_tuning best = default_tuning();
  double best_t = 0;
  sa_status st = SA_OK;
  // SA_TUNE_LOG set in the environment: one line per candidate on stderr.
  const bool log = std::getenv("SA_TUNE_LOG") != nullptr;
  auto trial = [&](const sa_tuning& t) -> sa_status {
    ctx->explicit_tuning = t;
    double ms = 0;
    sa_status e = time_build(ctx, d_texts, h_offsets, num_texts, d_sas, s, reps, &ms);
    if (e != SA_OK) return e;
    if (log) {
      std::fprintf(stderr,
                   "sa_tune: bits %u items %u block %u wgs/cu %u match %u round0_full %u "
                   "lazy_ratio %u: %.3f ms\n",
                   t.radix_bits, t.sort_items, t.sort_block, t.sort_wgs_per_cu, t.sort_match,
                   t.round0_full, t.lazy_ratio, ms);
      std::fflush(stderr);
    }
    if (best_t == 0 || ms < best_t) {
      best_t = ms;
      best = t;
    }
    return SA_OK;
  };
  // Stage 1: tile shape and persistent grid of the radix sweeps (the default
  // grid first, then explicit workgroups per CU).
  struct Shape {
    u32 items, block;
  };
  const Shape shapes[] = {{8, 256}, {12, 256}, {16, 256}, {20, 256}, {24, 256},
                          {4, 512}, {8, 512}, {12, 512}};
  const u32 wgs_set[] = {0, 1, 2, 3, 4};
  for (const Shape& sh : shapes) {
    for (u32 w : wgs_set) {
      if (st != SA_OK) break;
      sa_tuning t = default_tuning();
      t.sort_items = sh.items;
      t.sort_block = sh.block;
      t.sort_wgs_per_cu = w;
      if (w != 0 && int(w) == default_wgs_per_cu(int(sh.items), int(sh.block), false, kRadixBits))
        continue;  // same as w = 0
      st = trial(t);
    }
  }
  // Stage 2: radix digit width (6, 7 and 9 bits run with 512-thread
  // workgroups and ballot matching) at the default grid.
  struct Width {
    u32 rb, items;
  };
  const Width widths[] = {{6, 4}, {6, 8}, {6, 12}, {7, 4}, {7, 8}, {7, 12}, {9, 8}};
  for (const Width& wd : widths) {
    if (st != SA_OK) break;
    sa_tuning t = best;
    t.radix_bits = wd.rb;
    t.sort_items = wd.items;
    t.sort_block = 512;
    t.sort_match = 0;
    t.sort_wgs_per_cu = 0;
    st = trial(t);
  }
  // Stage 3: digit matching of the sweep (8-bit digits); stage 4: round-0 key
  // width; stage 5: the lazy-ISA threshold.
  if (st == SA_OK && best.radix_bits == u32(kRadixBits)) {
    sa_tuning t = best;
    t.sort_match = 1;
    st = trial(t);
  }
  if (st == SA_OK) {
    sa_tuning t = best;
    t.round0_full = 1 - best.round0_full;
    st = trial(t);
  }
  const u32 lazy_set[] = {3, 4, 16, 64};
  for (u32 lr : lazy_set) {
    if (st != SA_OK) break;
    if (lr == best.lazy_ratio) continue;
    sa_tuning t = best;
    t.lazy_ratio = lr;
    st = trial(t);
  }
  u32 code_bits = 0;
  if (st == SA_OK) {
    // One more build with the winner, for the code width of the entry.
    ctx->explicit_tuning = best;
    double ms = 0;
    st = time_build(ctx, d_texts, h_offsets, num_texts, d_sas, s, 1, &ms);
    code_bits = num_texts == 1 ? ctx->info.code_bits : 0;
  }
  ctx->tuning_explicit = was_explicit;
  ctx->trace = was_trace;
  ctx->recs.clear();
  ctx->event_used = 0;
  if (st != SA_OK) return st;
  TuneEntry e;
  e.arch = ctx->arch;
  e.mode = num_texts == 1 ? "single" : "batch";
  e.log2n = log2_floor(N);
  e.code_bits = code_bits;
  e.t = best;
  e.ms = best_t;
  tune_upsert(*ctx->tune, e);
  if (best_out) *best_out = best;
  if (best_ms) *best_ms = best_t;
  return SA_OK;
}

sa_status sa_tune_save(const sa_ctx* ctx, const char* path) {
  if (!ctx) return SA_EINVAL;
  if (!path) path = ctx->tune_path.empty() ? nullptr : ctx->tune_path.c_str();
  if (!path) return SA_EINVAL;
  static const TuneTable empty;
  return tune_save(path, ctx->tune ? *ctx->tune : empty);
}

sa_status sa_tune_lookup(const char* path, const char* arch, const char* mode, uint64_t n,
                         uint32_t code_bits, sa_tuning* out, int* found) {
  if (!path || !arch || !mode || !out || !found) return SA_EINVAL;
  if (std::strcmp(mode, "single") != 0 && std::strcmp(mode, "batch") != 0) return SA_EINVAL;
  *found = 0;
  TuneTable t;
  sa_status st = tune_load(path, t);
  if (st != SA_OK) return st;
  const TuneEntry* e = tune_lookup(t, arch, mode, log2_floor(n), code_bits);
  *out = e ? e->t : default_tuning();
  *found = e ? 1 : 0;
  return SA_OK;
}

}  // extern "C"
