// Internal host-side driver shared by the single-text, batched and serving
// paths: the context (workspace, plans, tracing) and the round building blocks.
#pragma once

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sa.h"
#include "kernels.h"

using namespace sa;

// Automatic ISA mode: lazy when at most 1/kLazyRatio of the suffixes survive
// round 0 (each later gather may then cost a binary search instead of every
// suffix costing a random 4-byte write).
constexpr u64 kLazyRatioDefault = 8;

// Tuning cache: one entry per (architecture, mode, log2 size, code bits).
constexpr const char* kTuneFormat = "sa_mi355x_tune/1";
struct TuneEntry {
  std::string arch;  // e.g. "gfx950"
  std::string mode;  // "single" or "batch"
  u32 log2n = 0;     // floor(log2 of the text or batch length)
  u32 code_bits = 0; // bits per character code of the tuned input (0: any)
  sa_tuning t{};
  double ms = 0;     // build time of the winner when tuned
};
struct TuneTable {
  std::vector<TuneEntry> entries;
};

// A captured later round (rounds run ahead of the host), keyed by everything
// its launch arguments depend on. A key is captured the second time it is
// seen, so that one-off builds never pay for capture.
struct GraphKey {
  u64 n, bound;
  const void* ptr[12];
  u32 knobs[12];
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec = nullptr;
  u32 seen = 0;
  u64 last_use = 0;
};

struct TraceRec {
  hipEvent_t start, stop;
  int kind;
  double bytes;      // algorithmic bytes, if known at launch
  int sort_slot;     // >= 0: bytes depend on the plan of this sort (pass `pass`)
  int pass;
  u64 count;
};

struct sa_ctx {
  int device = 0;
  u64 cap = 0;  // element capacity of the workspace
  u64* keysA = nullptr;
  u64* keysB = nullptr;
  u32* valsA = nullptr;
  u32* valsB = nullptr;
  u32* isa = nullptr;
  u32* live = nullptr;    // lazy ISA: bitmap of the positions whose ISA entry is set
  u32* act_idx = nullptr;
  u32* act_rank = nullptr;
  u64* act_ti = nullptr;  // batch survivors: (text << 32) | local position
  u64 act_ti_cap = 0;
  u64* toff = nullptr;    // batch text offsets on the device
  u64 toff_cap = 0;
  u64* status = nullptr;  // sort look-back: [tiles][radix]
  // Arrays of the difference cover builds, per (recursion depth, slot), kept
  // between builds so that repeated builds allocate nothing.
  std::vector<std::pair<void*, size_t>> level_bufs;
  // Sort-based pairing (sa_build_sorted_pairs): three item buffers.
  u64* pair_k[3] = {nullptr, nullptr, nullptr};
  u32* pair_v[3] = {nullptr, nullptr, nullptr};
  u64 pair_cap = 0;
  // Small control block: hist_in | hist_run | tickets | counters | plan | present | code.
  void* small = nullptr;
  u32* hist_in = nullptr;   // [passes][kChunks][radix] input-order chunk histograms
  u32* hist_run = nullptr;  // [passes][kChunks][radix] histograms fed forward by sweeps
  u32* tickets = nullptr;   // [kMaxPasses][kChunks] tile tickets
  u64* counters = nullptr;
  RoundCtl* rc = nullptr;   // rounds run from the device (follows the counters)
  u32* plan_log = nullptr;  // [kPlanLogRows][kPlanLogWords] (follows rc)
  SortCtl* ctl = nullptr;
  SortPlan* plan = nullptr;
  u32* present = nullptr;
  u16* code = nullptr;
  u64* sample = nullptr;  // lazy ISA: sampled round-0 sorted keys
  u32* stage_hist = nullptr;  // staged ISA writes: counts per (bucket, re-rank workgroup)
  // Pinned mirror of counters | rc | plan_log, refreshed by every readback.
  void* h_mirror = nullptr;
  u64* h_counters = nullptr;
  RoundCtl* h_rc = nullptr;
  u32* h_plans = nullptr;  // [kPlanLogRows][kPlanLogWords]
  u32 gen = 1;             // upper bound of ctl->gen_next (look-back generations)
  // Later rounds run ahead of the host: at most this many per readback
  // (0 = adaptive, doubling from 1), replayed from captured graphs unless
  // graphs are off (tuning) or tracing / the no-allocation call is active.
  u32 rounds_ahead = 0;
  bool graphs = true;
  bool graphs_blocked = false;
  hipStream_t cap_stream = nullptr;
  std::vector<GraphEntry> graph_cache;
  u64 graph_clock = 0;
  u64 graph_launches = 0;  // replays of captured rounds (diagnostics)
  int isa_mode = SA_ISA_AUTO;
  int sort_items = kSortItemsDefault;  // radix-sort items per thread (tile size)
  int sort_block = kSortBlockDefault;  // radix-sort workgroup size (256 or 512)
  int sort_wgs_per_cu = 0;             // persistent sweep workgroups per CU (0 = by tile size)
  int sort_match = 0;                  // sweep digit matching: 0 ballots, 1 LDS table
  int radix_bits = kRadixBits;         // radix-sort digit width
  int prefix_mult = 2;                 // 2: prefix doubling; 4: prefix quadrupling (sa_build)
  bool stage_isa = true;               // names of long single texts staged by position bucket
  int num_cus = 256;
  u64 lazy_ratio = kLazyRatioDefault;
  int round0_trim = 1;  // round-0 keys fill whole radix digits
  // Tuning: an explicit choice from sa_ctx_set_tuning wins; otherwise each
  // build looks its input up in the cache table (defaults when absent).
  bool tuning_explicit = false;
  sa_tuning explicit_tuning{};
  TuneTable* tune = nullptr;
  std::string tune_path;
  std::string arch;         // architecture name without feature suffixes
  u32 sigma_hint = 0;       // alphabet hint of the current sa_build (0: none)
  int tuned_from_cache = 0; // 1 if the last build took its knobs from the table
  bool trace = false;
  std::vector<TraceRec> recs;
  std::vector<hipEvent_t> event_pool;
  size_t event_used = 0;
  sa_kernel_stats stats[SA_KERNEL_KINDS];
  sa_build_info info;
};


namespace drv {

// Chunk histograms of one sort: passes x chunks x digits, for the digit width
// that needs the most words.
constexpr size_t hist_words_for(int rb) {
  return size_t(passes_for(64, rb)) * kChunks * (size_t(1) << rb);
}
constexpr size_t max_hist_words(int rb) {
  return rb > kRadixBitsMax ? 0
                            : (hist_words_for(rb) > max_hist_words(rb + 1) ? hist_words_for(rb)
                                                                             : max_hist_words(rb + 1));
}
constexpr size_t kChunkHistWords = max_hist_words(kRadixBitsMin);
constexpr size_t kTicketWords = size_t(kMaxPasses) * kChunks;
static_assert(SA_MAX_ROUNDS == kMaxRounds, "round logs");
constexpr size_t kSmallHist = (2 * kChunkHistWords + kTicketWords) * sizeof(u32);
constexpr size_t kClearWords = 2 * kChunkHistWords + kTicketWords;  // cleared by sort_begin
// The readback span: counters | RoundCtl | plan log, contiguous.
constexpr size_t kSmallCounters = size_t(kCtrCount) * sizeof(u64);
constexpr size_t kSmallRoundCtl = sizeof(RoundCtl);
constexpr int kPlanFlagWords = kPlanLogWords;  // skip, src, iota, final_buf
constexpr size_t kSmallPlanLog = (size_t(kPlanLogRows) * kPlanFlagWords * sizeof(u32) + 255) /
                                 256 * 256;
constexpr size_t kMirrorBytes = kSmallCounters + kSmallRoundCtl + kSmallPlanLog;
constexpr size_t kSmallCtl = 256;
constexpr size_t kSmallPlan = (sizeof(SortPlan) + 255) / 256 * 256;
constexpr size_t kSmallPresent = 256 * sizeof(u32);
constexpr size_t kSmallCode = 256 * sizeof(u16);
constexpr size_t kSmallSample = size_t(kLazySamples) * sizeof(u64);
constexpr size_t kSmallStage = size_t(kStageBuckets) * kStageMaxWgs * sizeof(u32);
constexpr size_t kSmallBytes = kSmallHist + kMirrorBytes + kSmallCtl + kSmallPlan + kSmallPresent +
                               kSmallCode + kSmallSample + kSmallStage;
static_assert(kSmallCounters % 8 == 0 && kSmallRoundCtl % 8 == 0, "mirror alignment");
static_assert(sizeof(SortCtl) <= kSmallCtl, "control block");


template <typename T>
bool dev_alloc(T** p, u64 count) {
  if (hipMalloc(reinterpret_cast<void**>(p), std::max<u64>(count, 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return false;
  }
  return true;
}

u64 sort_status_words(u64 cap);
int bits_of(u64 v);
void free_workspace(sa_ctx* c);
sa_status ensure_workspace(sa_ctx* c, u64 n);
// Reserves `count` look-back generations; clears the status words and
// restarts the device counter first when the 22-bit tags would wrap.
void reserve_gens(sa_ctx* c, u32 count, hipStream_t s);
void bind_small(sa_ctx* c, char* p);
// Initial control words of a freshly allocated control block (synchronous).
sa_status init_small(char* p);
void drop_graphs(sa_ctx* c);
void free_pair_workspace(sa_ctx* c);
// The difference cover builds' array `slot` of recursion depth `depth`, at
// least `bytes` long (grown on demand, owned by the context).
void* level_buf(sa_ctx* c, u32 depth, u32 slot, size_t bytes);
void free_level_bufs(sa_ctx* c);
constexpr u32 kLevelSlots = 24;
template <typename T>
bool level_alloc(sa_ctx* c, u32 depth, u32 slot, u64 count, T** p) {
  *p = static_cast<T*>(level_buf(c, depth, slot, std::max<u64>(count, 1) * sizeof(T)));
  return *p != nullptr;
}
// Suffix array of a string of m names (values 1..max_sym, 0 past the end) by
// DC3, at recursion depth `depth` (dc3.hip; DC7 recurses through it).
sa_status dc3_names(sa_ctx* c, const u32* x, u64 m, u64 max_sym, u32* sa, u32 depth,
                    hipStream_t s);
hipEvent_t take_event(sa_ctx* c);

// Brackets one launch with events when tracing.
struct Tracer {
  sa_ctx* c;
  hipStream_t s;
  TraceRec rec{};
  bool on;
  Tracer(sa_ctx* ctx, hipStream_t st, int kind, double bytes, int sort_slot = -1, int pass = 0,
         u64 count = 0)
      : c(ctx), s(st), on(ctx->trace) {
    if (!on) return;
    rec.kind = kind;
    rec.bytes = bytes;
    rec.sort_slot = sort_slot;
    rec.pass = pass;
    rec.count = count;
    rec.start = take_event(c);
    rec.stop = take_event(c);
    if (!rec.start || !rec.stop) {
      on = false;
      return;
    }
    (void)hipEventRecord(rec.start, s);
  }
  ~Tracer() {
    if (!on) return;
    (void)hipEventRecord(rec.stop, s);
    c->recs.push_back(rec);
  }
};

void collect_trace(sa_ctx* c);

// Ping-pong buffers of one sort: input in (kA, vA), output in A or B.
struct Bufs {
  u64* kA;
  u64* kB;
  u32* vA;
  u32* vB;
};

Bufs full_bufs(sa_ctx* c);
int default_wgs_per_cu(int items, int block, bool table, int rb);
// Radix passes that cover `bits` key bits at the context's digit width.
inline int npass_for(const sa_ctx* c, int bits) { return passes_for(bits, c->radix_bits); }
// A sort in two parts: begin_sort sets the control words (count = *dev_count,
// else `bound`; with rc it starts a device-driven round); sort_passes runs the
// histogram, the plan (flags to plan-log row `log_row`, rc->round when < 0)
// and the sweeps. `bound` >= the count sizes the launch grids. With
// reserve == false the caller has reserved the generations already.
void begin_sort(sa_ctx* c, u64 bound, const u64* dev_count, RoundCtl* rc, int npass, bool reserve,
                hipStream_t s, u64 dense_n = 0, int log2a = 1);
void sort_passes(sa_ctx* c, const Bufs& bf, u64 bound, int npass, int vals_present, int log_row,
                 u64 trace_count, hipStream_t s);
// A sort of `count` pairs known on the host.
void run_sort(sa_ctx* c, const Bufs& bf, u64 count, int npass, int vals_present, int slot,
              hipStream_t s);
// Re-rank of the current sort (ctl->count elements, at most `bound`).
void run_rerank(sa_ctx* c, const Bufs& bf, const RerankArgs& args, u32* d_sa, u64 bound,
                u64 trace_count, hipStream_t s);
u32 stream_grid(const sa_ctx* c, u64 bound, u32 per_block);
// Workgroups of 256 threads for a grid-stride kernel whose threads each make
// scattered 4-byte writes: about four per CU. Scattered writes run fastest with
// few in flight (twice as many take about twice as long).
u32 scatter_grid(const sa_ctx* c, u64 bound);
RerankArgs single_args(u64 count, u64 n, int b, int mode);
sa_status readback(sa_ctx* c, hipStream_t s);
u32 passes_run(const sa_ctx* c, int slot, int npass);
u32 final_buf_of(const sa_ctx* c, int slot);
sa_status build_rounds(sa_ctx* c, const u8* text, u64 n, u32 max_rounds, u32* d_sa, u32* d_isa,
                       hipStream_t s);
// Settles trace records after a build: collected on success, dropped on error.
void settle_trace(sa_ctx* c, sa_status st);
sa_status build_batch_impl(sa_ctx* c, const u8* text, const u64* h_off, u32 T, u32* d_sa,
                           hipStream_t s);

// Per-slot tables of the multi-text engine (multi.hip), in one allocation.
struct TableLayout {
  size_t o_base, o_len, o_h, o_start, o_r0, o_nt, o_no, o_nc;  // uploaded each round
  size_t up_bytes;                                     // extent of the uploaded part
  size_t o_code, o_pres, o_wc, o_surv;
  size_t bytes;
};
TableLayout table_layout(u32 nslots);

// Tuning (tune.hip).
bool tuning_valid(const sa_tuning& t);
sa_tuning default_tuning();
void apply_tuning(sa_ctx* c, const sa_tuning& t);
sa_tuning current_tuning(const sa_ctx* c);
sa_status tune_load(const char* path, TuneTable& out);
void resolve_tuning(sa_ctx* c, const char* mode, u64 n, u32 code_bits);

}  // namespace drv
