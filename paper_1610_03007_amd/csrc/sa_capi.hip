// Context, round driver and C ABI of the gfx950 suffix-array library.
//
// The driver runs the loop of prefix doubling with discarding (Section 2.1,
// Alg. 5): round 0 sorts keys of c packed characters; each later round sorts
// only the suffixes whose name is not yet unique, by the name pair (own name,
// name of the suffix h positions on), with h doubling every round, until no
// suffix is left. One 8-byte readback per round tells the host how many
// suffixes remain.

#include <atomic>
#include <mutex>
#include "driver.h"

namespace drv {

// Look-back statuses: one per digit of every tile. Tiles of 256-digit sorts
// have at least kSortTileMin pairs and those of 512-digit sorts at least
// 2 * kSortTileMin, so 256 words per kSortTileMin pairs (and one tile of
// slack for the rounding) hold either.
u64 sort_status_words(u64 cap) { return (ceil_div(cap, kSortTileMin) + 1) * kRadix; }

int bits_of(u64 v) { return v == 0 ? 0 : 64 - __builtin_clzll(v); }

void free_workspace(sa_ctx* c) {
  (void)hipFree(c->keysA);
  (void)hipFree(c->keysB);
  (void)hipFree(c->valsA);
  (void)hipFree(c->valsB);
  (void)hipFree(c->isa);
  (void)hipFree(c->live);
  (void)hipFree(c->act_idx);
  (void)hipFree(c->status);
  (void)hipFree(c->act_ti);
  c->act_ti = nullptr;
  c->act_ti_cap = 0;
  c->keysA = c->keysB = nullptr;
  c->valsA = c->valsB = c->isa = c->act_idx = c->act_rank = c->live = nullptr;
  c->status = nullptr;
  c->cap = 0;
}

sa_status ensure_workspace(sa_ctx* c, u64 n) {
  if (n <= c->cap) return SA_OK;
  free_workspace(c);
  u64 cap = std::max<u64>(n, 1 << 16);
  bool ok = dev_alloc(&c->keysA, cap) && dev_alloc(&c->keysB, cap) && dev_alloc(&c->valsA, cap) &&
            dev_alloc(&c->valsB, cap) && dev_alloc(&c->isa, cap) && dev_alloc(&c->act_idx, 2 * cap) &&
            dev_alloc(&c->live, ceil_div(cap, 32)) &&
            dev_alloc(&c->status, sort_status_words(cap));
  if (!ok) {
    free_workspace(c);
    return SA_ENOMEM;
  }
  // The active list's ranks follow its positions in the same allocation, so
  // that a quadrupling round can use both as one u64 array.
  c->act_rank = c->act_idx + cap;
  // The status array starts cleared; generations then keep it valid without
  // further clearing.
  if (hipMemset(c->status, 0, sort_status_words(cap) * sizeof(u64)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    free_workspace(c);
    return SA_EDEVICE;
  }
  // Captured rounds name the old buffers.
  drop_graphs(c);
  c->cap = cap;
  return SA_OK;
}

void reserve_gens(sa_ctx* c, u32 count, hipStream_t s) {
  if (u64(c->gen) + count + 1 >= kGenMask) {
    launch_fill_u64(c->status, sort_status_words(c->cap), 0, s);
    launch_sort_gen_reset(c->ctl, s);
    c->gen = 1;
  }
  c->gen += count;
}

sa_status init_small(char* p) {
  // Everything zero, then the generation counter at 1.
  SortCtl ctl{};
  ctl.gen_next = 1;
  if (hipMemset(p, 0, kSmallBytes) != hipSuccess ||
      hipMemcpy(p + kSmallHist + kMirrorBytes, &ctl, sizeof(ctl), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    return SA_EDEVICE;
  }
  return SA_OK;
}

void* level_buf(sa_ctx* c, u32 depth, u32 slot, size_t bytes) {
  const size_t k = size_t(depth) * kLevelSlots + slot;
  if (c->level_bufs.size() <= k) c->level_bufs.resize(k + 1, {nullptr, 0});
  auto& e = c->level_bufs[k];
  if (e.second >= bytes) return e.first;
  (void)hipFree(e.first);
  e = {nullptr, 0};
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  e = {p, bytes};
  return p;
}

void free_level_bufs(sa_ctx* c) {
  for (auto& e : c->level_bufs) (void)hipFree(e.first);
  c->level_bufs.clear();
}

void drop_graphs(sa_ctx* c) {
  for (GraphEntry& e : c->graph_cache)
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
  c->graph_cache.clear();
}

hipEvent_t take_event(sa_ctx* c) {
  if (c->event_used == c->event_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->event_pool.push_back(e);
  }
  return c->event_pool[c->event_used++];
}

void collect_trace(sa_ctx* c) {
  for (const TraceRec& r : c->recs) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    double bytes = r.bytes;
    if (r.sort_slot >= 0) {
      const u32* f = c->h_plans + size_t(r.sort_slot) * kPlanFlagWords;
      const bool skip = f[r.pass] != 0;
      const bool iota = f[2 * kMaxPasses + r.pass] != 0;
      // A skipped pass returns at once: counted as a launch that moved nothing.
      bytes = skip ? 0.0 : double(r.count) * (iota ? 20.0 : 24.0);
    }
    sa_kernel_stats& st = c->stats[r.kind];
    st.launches += 1;
    st.ms += ms;
    st.bytes += bytes;
  }
  c->recs.clear();
  c->event_used = 0;
}

Bufs full_bufs(sa_ctx* c) { return Bufs{c->keysA, c->keysB, c->valsA, c->valsB}; }

// Workgroups of a grid-stride launch over at most `bound` items, per_block
// items per workgroup: enough to fill the CUs, never more than the items.
u32 stream_grid(const sa_ctx* c, u64 bound, u32 per_block) {
  const u64 want = std::max<u64>(1, ceil_div(bound, per_block));
  return u32(std::min<u64>(want, u64(c->num_cus) * 16));
}

u32 scatter_grid(const sa_ctx* c, u64 bound) {
  const u64 want = std::max<u64>(1, ceil_div(bound, 256));
  return u32(std::min<u64>(want, u64(c->num_cus) * 4));
}

// Sweep workgroups one CU holds at once for each tile shape (register and LDS
// limits of the kernel instances).
int default_wgs_per_cu(int items, int block, bool table, int rb) {
  // The runtime's occupancy figure for the shape, cached per shape; if the
  // query fails, what one CU's 160 KB of LDS holds: the key tile, the per-wave
  // digit counts (16 bits), the 16-bit chunk histograms of the next sweep, the
  // match table if any and about 4 KB of small arrays.
  static std::atomic<int> cache[kRadixBitsMax - kRadixBitsMin + 1][2][2][32];
  const int ri = std::min(std::max(rb, kRadixBitsMin), kRadixBitsMax) - kRadixBitsMin;
  const int bi = block == 512 ? 1 : 0;
  const int ii = items & 31;
  const int ti = table ? 1 : 0;
  int n = cache[ri][ti][bi][ii].load(std::memory_order_relaxed);
  if (n > 0) return n;
  n = onesweep_wgs_per_cu(items, block, table, rb);
  if (n <= 0) {
    const int radix = 1 << rb;
    const int lds = block * items * 8 + (block / kWave / 2) * radix * 4 + kChunks * radix * 2 +
                    (table ? (block / kWave) * radix * 8 : 0) + radix * 12 + 1024;
    n = (160 * 1024) / lds;
    if (n < 1) n = 1;
    return n;
  }
  cache[ri][ti][bi][ii].store(n, std::memory_order_relaxed);
  return n;
}

void begin_sort(sa_ctx* c, u64 bound, const u64* dev_count, RoundCtl* rc, int npass, bool reserve,
                hipStream_t s, u64 dense_n, int log2a) {
  if (reserve) reserve_gens(c, u32(npass), s);
  Tracer t(c, s, SA_KERNEL_OTHER, 0);
  static_assert(kCtrSortTiles < kCtrActive && kCtrKeyOr < kCtrActive && kCtrKeyNot < kCtrActive,
                "sort_begin clears the sort's counters");
  launch_sort_begin(c->ctl, rc, bound, dev_count, npass, dense_n, log2a, c->hist_in, kClearWords,
                    c->counters, s);
}

// Sorts (kA, vA or generated values) by the low 8*npass bits. The sorted pairs
// end in the buffer named by plan->final_buf.
void sort_passes(sa_ctx* c, const Bufs& bf, u64 bound, int npass, int vals_present, int log_row,
                 u64 trace_count, hipStream_t s) {
  const u32 tile = u32(c->sort_items * c->sort_block);
  const bool table = c->sort_match == 1;
  const u32 hgrid = radix_histogram_grid(bound, tile);
  {
    Tracer t(c, s, SA_KERNEL_HISTOGRAM, double(trace_count) * 8.0);
    launch_radix_histogram(bf.kA, c->ctl, tile, hgrid, c->hist_in, c->counters, c->radix_bits, s);
  }
  {
    Tracer t(c, s, SA_KERNEL_OTHER, 0);
    launch_radix_plan(c->ctl, c->counters, npass, vals_present, c->plan, c->plan_log, log_row,
                      c->rc, c->radix_bits, s);
    launch_radix_histogram_first(bf.kA, c->ctl, tile, hgrid, c->plan, c->hist_in, c->radix_bits,
                                 s);
  }
  // Persistent sweep workgroups: what the CUs hold, at most one per tile of
  // the bound, at least one per chunk.
  const u64 tiles = ceil_div(std::max<u64>(bound, 1), tile);
  const int per_cu = c->sort_wgs_per_cu > 0
                         ? c->sort_wgs_per_cu
                         : default_wgs_per_cu(c->sort_items, c->sort_block, table, c->radix_bits);
  u64 grid = std::min<u64>(tiles, u64(c->num_cus) * u64(per_cu));
  grid = std::max<u64>(grid, u64(kChunks));
  for (int p = 0; p < npass; ++p) {
    Tracer t(c, s, SA_KERNEL_SORT_PASS, 0, log_row, p, trace_count);
    launch_onesweep_pass(bf.kA, bf.kB, bf.vA, bf.vB, c->ctl, p, c->plan, c->hist_in, c->hist_run,
                         c->tickets, c->status, c->counters, c->sort_items, c->sort_block, table,
                         c->radix_bits, u32(grid), s);
  }
}

void run_sort(sa_ctx* c, const Bufs& bf, u64 count, int npass, int vals_present, int slot,
              hipStream_t s) {
  begin_sort(c, count, nullptr, nullptr, npass, true, s);
  sort_passes(c, bf, count, npass, vals_present, slot, count, s);
}

void run_rerank(sa_ctx* c, const Bufs& bf, const RerankArgs& args, u32* d_sa, u64 bound,
                u64 trace_count, hipStream_t s) {
  const double count = double(trace_count);
  // 12 bytes read per element; 4 written (ISA, SA or survivor name) plus 4 for a
  // survivor's position, counted as 4 per element either way.
  double bytes = count * 16.0 - ((args.mode & kRerankScatterIsa) ? 0.0 : 4.0 * count);
  if (args.mode & kRerankIsaOnly) bytes = count * 16.0;
  Tracer t(c, s, (args.mode & kRerankIsaOnly) ? SA_KERNEL_ISA_SCATTER : SA_KERNEL_RERANK, bytes);
  const u32 grid = u32(std::min<u64>(std::max<u64>(1, ceil_div(bound, kRerankTile)),
                                     u64(c->num_cus) * rerank_wgs_per_cu(args.tie != 0)));
  // Names of one long text go through the staged writes (when the device
  // count turns out large enough): its ISA is far larger than the caches.
  RerankArgs a = args;
  const bool stage = (a.mode & kRerankScatterIsa) && !(a.mode & (kRerankPairOut | kRerankEmit)) &&
                     !a.tbase && a.n >= kStageMinN && grid <= kStageMaxWgs && c->stage_isa;
  if (stage) {
    a.stage_a = bf.kA;
    a.stage_b = bf.kB;
    a.stage_hist = c->stage_hist;
    a.stage_w = u32(ceil_div(a.n, u64(kStageBuckets)));
  }
  launch_rerank_compact(bf.kA, bf.kB, bf.vA, bf.vB, c->plan, a, c->ctl, c->isa, d_sa,
                        a.tbase ? nullptr : c->act_idx, a.tbase ? c->act_ti : nullptr,
                        c->act_rank, c->counters, grid, s);
  if (stage)
    launch_stage_isa(bf.kA, bf.kB, c->plan, c->ctl, c->stage_hist, grid, a.stage_w, a.n, c->isa,
                     c->counters, u32(c->num_cus) * 4, s);
}

// Re-rank arguments of a single text: round 0 (one group, every rank 1) or a
// later round with (rank << b | next rank) keys.
RerankArgs single_args(u64 count, u64 n, int b, int mode) {
  RerankArgs a{};
  a.count = count;
  a.n = n;
  a.gshift = b > 0 ? b : 64;
  a.rshift = b;
  a.rmask = b > 0 ? ~u64(0) : 0;
  a.idshift = 0;
  a.mode = mode;
  a.tbase = nullptr;
  a.tlen = nullptr;
  a.tround0 = nullptr;
  return a;
}

sa_status readback(sa_ctx* c, hipStream_t s) {
  // counters | rc | plan log in one copy.
  if (hipMemcpyAsync(c->h_mirror, c->counters, kMirrorBytes, hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return SA_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return SA_EDEVICE;
  if (hipGetLastError() != hipSuccess) return SA_EDEVICE;
  if (c->h_counters[kCtrError] != 0) return SA_EDEVICE;
  return SA_OK;
}

u32 passes_run(const sa_ctx* c, int slot, int npass) {
  const u32* f = c->h_plans + size_t(slot) * kPlanFlagWords;
  u32 r = 0;
  for (int p = 0; p < npass; ++p) r += f[p] == 0;
  return r;
}

u32 final_buf_of(const sa_ctx* c, int slot) {
  return c->h_plans[size_t(slot) * kPlanFlagWords + 3 * kMaxPasses];
}

// Everything one later round of a single text reads: the same for every
// round of a build, so that a captured round replays unchanged.
struct LaterRound {
  u64 n, bound;
  u64 dense_n;  // n when dense rounds are allowed (the ISA holds every name), else 0
  int b, npass;
  bool lazy;
  bool quad;    // prefix quadrupling: rank quadruples, two sorts per round (needs the eager ISA)
  Bufs bufs;
  const u8* text;
  const u64* keys0;
  u32* d_sa;
};

// One later round (Alg. 5 loop body): the round's count is the last re-rank's
// survivor count, read on the device; with none left every kernel returns at
// once. log_row: the plan-log row (the round index), or -1 to take it from the
// device. trace_count: the count, when the host knows it (tracing).
// A quadrupling round (Section 2.1, prefix quadrupling): the rank quadruple
// (r0, r1, r2, r3) is sorted as two words, the low one first (see
// launch_pack_quad_lo), and renamed with the low word's run names as ties.
// pk (u64 per element) spans the active-list arrays, which the round reads
// only before it is written and writes only after it is consumed.
void enqueue_quad_round(sa_ctx* c, const LaterRound& L, bool reserve, int log_row,
                        u64 trace_count, bool trace_dense, hipStream_t s) {
  u64* pk = reinterpret_cast<u64*>(c->act_idx);
  const u32 grid = stream_grid(c, L.bound, 256);
  begin_sort(c, L.bound, c->counters + kCtrActive, c->rc, L.npass, reserve, s, L.dense_n, 2);
  {
    // Two names in (gathered unless dense), the low key and the position out.
    Tracer t(c, s, SA_KERNEL_PACK_PAIRS, double(trace_count) * (trace_dense ? 16.0 : 20.0));
    launch_pack_quad_lo(c->act_idx, c->ctl, c->rc, L.n, L.b, c->isa, L.bufs.kA, L.bufs.vA, grid,
                        s);
  }
  sort_passes(c, L.bufs, L.bound, L.npass, 1, log_row, trace_count, s);
  {
    RerankArgs a = single_args(L.bound, L.n, 0, kRerankPairOut);
    a.pair_out = pk;
    run_rerank(c, L.bufs, a, L.d_sa, L.bound, trace_count, s);
  }
  {
    // Position in; two gathered names in, the high key out.
    Tracer t(c, s, SA_KERNEL_PACK_PAIRS, double(trace_count) * 24.0);
    launch_pack_quad_hi(pk, c->ctl, c->rc, L.n, L.b, c->isa, L.bufs.kA, c->counters, grid, s);
  }
  // The high-word sort: the same count, values generated (the low-sorted index).
  begin_sort(c, L.bound, &c->ctl->count, nullptr, L.npass, reserve, s, 0, 1);
  sort_passes(c, L.bufs, L.bound, L.npass, 0,
              log_row >= 0 ? log_row + kPlanRowSecond : kLogRowRoundSecond, trace_count, s);
  {
    // Index in and in place out; a gathered 8-byte pair; the tie word out.
    Tracer t(c, s, SA_KERNEL_OTHER, double(trace_count) * 20.0);
    launch_quad_permute(c->ctl, c->plan, pk, L.bufs.vA, L.bufs.vB, c->counters, grid, s);
  }
  RerankArgs a = single_args(L.bound, L.n, L.b, kRerankScatterIsa);
  a.tie = 1;
  run_rerank(c, L.bufs, a, L.d_sa, L.bound, trace_count, s);
}

void enqueue_later_round(sa_ctx* c, const LaterRound& L, bool reserve, int log_row,
                         u64 trace_count, bool trace_dense, hipStream_t s) {
  if (L.quad) {
    enqueue_quad_round(c, L, reserve, log_row, trace_count, trace_dense, s);
    return;
  }
  begin_sort(c, L.bound, c->counters + kCtrActive, c->rc, L.npass, reserve, s, L.dense_n, 1);
  {
    // A dense round reads two names and writes a key per suffix (16 bytes);
    // otherwise index, rank and the gathered name in, key and value out.
    Tracer t(c, s, SA_KERNEL_PACK_PAIRS, double(trace_count) * (trace_dense ? 16.0 : 24.0));
    const u32 grid = stream_grid(c, L.bound, 256);
    if (L.lazy)
      launch_pack_pairs_lazy(c->act_idx, c->act_rank, c->ctl, c->rc, L.n, L.b, c->isa, L.text,
                             c->code, c->counters, L.keys0, c->sample, c->live, L.bufs.kA,
                             L.bufs.vA, grid, s);
    else
      launch_pack_pairs(c->act_idx, c->act_rank, c->ctl, c->rc, L.n, L.b, c->isa, L.bufs.kA,
                        L.bufs.vA, grid, s);
  }
  sort_passes(c, L.bufs, L.bound, L.npass, 1, log_row, trace_count, s);
  run_rerank(c, L.bufs, single_args(L.bound, L.n, L.b, kRerankScatterIsa), L.d_sa, L.bound,
             trace_count, s);
}

GraphKey later_key(const sa_ctx* c, const LaterRound& L) {
  GraphKey k;
  std::memset(&k, 0, sizeof(k));
  k.n = L.n;
  k.bound = L.bound | (L.dense_n ? u64(1) << 63 : 0);
  const void* p[12] = {L.bufs.kA, L.bufs.kB, L.bufs.vA, L.bufs.vB, L.text, L.keys0, L.d_sa,
                       c->isa, c->act_idx, c->small, c->status, c->live};
  std::memcpy(k.ptr, p, sizeof(p));
  const u32 knobs[11] = {u32(L.b),           u32(L.npass),           L.lazy ? 1u : 0u,
                         u32(c->sort_items), u32(c->sort_block),     u32(c->sort_match),
                         u32(c->sort_wgs_per_cu), u32(c->num_cus),   u32(c->radix_bits),
                         L.quad ? 1u : 0u,   c->stage_isa ? 1u : 0u};
  std::memcpy(k.knobs, knobs, sizeof(knobs));
  return k;
}

// The captured form of L's round, if its key has been seen before (captured
// now on the second sighting); nullptr: launch directly.
hipGraphExec_t later_graph(sa_ctx* c, const LaterRound& L) {
  constexpr size_t kMaxGraphs = 8;
  const GraphKey key = later_key(c, L);
  c->graph_clock += 1;
  GraphEntry* e = nullptr;
  for (GraphEntry& g : c->graph_cache)
    if (std::memcmp(&g.key, &key, sizeof(key)) == 0) e = &g;
  if (!e) {
    if (c->graph_cache.size() >= kMaxGraphs) {
      auto lru = std::min_element(
          c->graph_cache.begin(), c->graph_cache.end(),
          [](const GraphEntry& a, const GraphEntry& b) { return a.last_use < b.last_use; });
      if (lru->exec) (void)hipGraphExecDestroy(lru->exec);
      c->graph_cache.erase(lru);
    }
    GraphEntry ne;
    ne.key = key;
    c->graph_cache.push_back(ne);
    e = &c->graph_cache.back();
  }
  e->last_use = c->graph_clock;
  e->seen += 1;
  if (e->exec || e->seen < 2) return e->exec;
  if (!c->cap_stream &&
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    c->cap_stream = nullptr;
    return nullptr;
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  enqueue_later_round(c, L, false, -1, 0, false, c->cap_stream);
  if (hipStreamEndCapture(c->cap_stream, &g) != hipSuccess || !g) {
    (void)hipGetLastError();
    return nullptr;
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    exec = nullptr;
  }
  (void)hipGraphDestroy(g);
  e->exec = exec;
  return exec;
}

sa_status build_rounds(sa_ctx* c, const u8* text, u64 n, u32 max_rounds, u32* d_sa, u32* d_isa,
                       hipStream_t s) {
  std::memset(&c->info, 0, sizeof(c->info));
  c->info.n = n;
  if (n == 0) return SA_OK;
  if (!text || !d_sa) return SA_EINVAL;
  if (n >= (u64(1) << 32)) return SA_ETOOBIG;
  if (hipSetDevice(c->device) != hipSuccess) return SA_EDEVICE;
  resolve_tuning(c, "single", n,
                 c->sigma_hint && c->sigma_hint < 256 ? u32(bits_of(c->sigma_hint)) : 0);
  sa_status st = ensure_workspace(c, n);
  if (st != SA_OK) return st;

  // Round 0: alphabet, packed keys, full sort, names, discard. The ISA is not
  // written yet; every sorted position's rank goes to the spare value buffer.
  const Bufs full = full_bufs(c);
  {
    Tracer t(c, s, SA_KERNEL_OTHER, 0);
    launch_fill_u64(c->counters, kCtrCount, 0, s);
    launch_fill_u64(reinterpret_cast<u64*>(c->rc), sizeof(RoundCtl) / 8, 0, s);
    launch_fill_u64(reinterpret_cast<u64*>(c->present), 256 / 2, 0, s);
  }
  {
    Tracer t(c, s, SA_KERNEL_OTHER, double(n));
    launch_byte_presence(text, n, c->present, s);
    launch_alphabet_codes(c->present, c->code, c->counters, c->round0_trim, 0, c->radix_bits, s);
  }
  {
    Tracer t(c, s, SA_KERNEL_PACK_TEXT, double(n) * 9.0);
    launch_pack_text(text, n, c->code, c->counters, c->keysA, s);
  }
  const int npass0 = npass_for(c, 64);
  run_sort(c, full, n, npass0, 0, 0, s);
  run_rerank(c, full, single_args(n, n, 0, 0), d_sa, n, n, s);
  st = readback(c, s);
  if (st != SA_OK) return st;

  sa_build_info& info = c->info;
  info.sigma = u32(c->h_counters[kCtrSigma]);
  info.code_bits = u32(c->h_counters[kCtrCodeBits]);
  info.chars0 = u32(c->h_counters[kCtrChars]);
  info.rounds = 1;
  info.active[0] = n;
  info.key_bits[0] = info.code_bits * info.chars0;
  info.passes_run[0] = passes_run(c, 0, npass0);
  const u64 chars0 = info.chars0;
  info.prefix_len = chars0;
  u64 active = c->h_counters[kCtrActive];

  // ISA after round 0: eager scatter, or lazy (survivors only) when few
  // suffixes survive and the later rounds' buffers fit in the spare keys.
  const u32 f0 = final_buf_of(c, 0);
  const u64* keys0 = f0 ? c->keysB : c->keysA;
  u64* spare = f0 ? c->keysA : c->keysB;
  // Later-round buffers are carved at 256-byte boundaries (vector accesses).
  const u64 a1 = (std::max<u64>(active, 1) + 63) / 64 * 64;
  const bool fits = a1 * 24 <= n * 8;
  // Quadrupling reads the names of positions i .. i + 3h from the ISA
  // directly, so it takes the eager form.
  const bool quad = c->prefix_mult == 4;
  bool lazy = false;
  if (quad)
    lazy = false;
  else if (c->isa_mode == SA_ISA_LAZY)
    lazy = fits;
  else if (c->isa_mode == SA_ISA_AUTO)
    lazy = fits && active * c->lazy_ratio <= n;
  info.lazy_isa = lazy ? 1u : 0u;
  if (active > 0 || d_isa) {
    if (lazy) {
      Tracer t(c, s, SA_KERNEL_OTHER, double(n) / 8.0 + double(active) * 12.0);
      launch_fill_u32(c->live, ceil_div(n, 32), 0, s);
      launch_isa_scatter_list(c->act_idx, c->act_rank, active, n, c->isa, c->live, s);
      launch_lazy_sample(keys0, n, c->sample, s);
    } else {
      run_rerank(c, full, single_args(n, n, 0, kRerankScatterIsa | kRerankIsaOnly), d_sa, n, n,
                 s);
    }
  }
  // Later rounds sort at most `active` pairs; in lazy mode their buffers are
  // carved out of the spare keys so that the round-0 sorted keys stay intact.
  LaterRound L;
  L.n = n;
  L.bound = std::max<u64>(active, 1);
  // Dense rounds read the name of every position, so only the eager ISA has them.
  L.dense_n = lazy ? 0 : n;
  L.b = bits_of(n);  // ranks and second ranks are <= n
  L.npass = npass_for(c, 2 * L.b);
  L.lazy = lazy;
  L.quad = quad;
  L.bufs = full;
  if (lazy) {
    L.bufs.kA = spare;
    L.bufs.kB = spare + a1;
    L.bufs.vA = reinterpret_cast<u32*>(spare + 2 * a1);
    L.bufs.vB = L.bufs.vA + a1;
  }
  L.text = text;
  L.keys0 = keys0;
  L.d_sa = d_sa;

  // Later rounds, run ahead of the host: up to `ahead` rounds are enqueued
  // before the survivor count is read back (1, 2, 4, ... unless fixed by the
  // tuning); a round that finds no survivor does nothing. Tracing runs one
  // round per readback so that every launch's count is known.
  const bool trace = c->trace;
  const bool use_graphs = c->graphs && !c->graphs_blocked && !trace;
  u32 ahead = c->rounds_ahead ? c->rounds_ahead : 1;
  u32 done = 0;  // later rounds run so far
  while (active > 0 && (max_rounds == 0 || info.rounds < max_rounds)) {
    u32 todo = trace ? 1 : ahead;
    if (max_rounds) todo = std::min<u32>(todo, max_rounds - info.rounds);
    todo = std::min<u32>(todo, u32(SA_MAX_ROUNDS - 1) - done);
    if (todo == 0) return SA_EDEVICE;  // cannot happen for n < 2^32
    hipGraphExec_t exec = use_graphs ? later_graph(c, L) : nullptr;
    if (exec) {
      reserve_gens(c, u32(L.npass) * todo * (quad ? 2u : 1u), s);
      for (u32 r = 0; r < todo; ++r)
        if (hipGraphLaunch(exec, s) != hipSuccess) return SA_EDEVICE;
      c->graph_launches += todo;
      info.graph_rounds += todo;
    } else {
      // With tracing (one round per readback) the host knows the round's count.
      const bool dense = L.dense_n && 4 * active >= 3 * L.dense_n;
      for (u32 r = 0; r < todo; ++r)
        enqueue_later_round(c, L, true, trace ? int(done + 1 + r) : -1,
                            trace ? (dense ? n : active) : 0, dense, s);
    }
    st = readback(c, s);
    if (st != SA_OK) return st;
    const u32 now = c->h_rc->round;
    if (now <= done || now > done + todo) return SA_EDEVICE;
    info.dense_rounds = c->h_rc->dense;
    for (u32 k = done + 1; k <= now; ++k) {
      info.active[k] = c->h_rc->active[k];
      info.key_bits[k] = u32((quad ? 4 : 2) * L.b);
      info.passes_run[k] = passes_run(c, int(k), L.npass) +
                           (quad ? passes_run(c, int(k) + kPlanRowSecond, L.npass) : 0u);
    }
    done = now;
    info.rounds = 1 + done;
    info.prefix_len = chars0 << ((quad ? 2 : 1) * done);
    active = c->h_counters[kCtrActive];
    if (!c->rounds_ahead) ahead = std::min<u32>(2 * ahead, 16);
  }
  if (d_isa) {
    if (lazy)
      launch_isa_complete(c->isa, n, text, c->code, c->counters, keys0, c->sample, c->live, s);
    if (hipMemcpyAsync(d_isa, c->isa, n * sizeof(u32), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return SA_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return SA_EDEVICE;
    if (hipGetLastError() != hipSuccess) return SA_EDEVICE;
  }
  return SA_OK;
}

void settle_trace(sa_ctx* c, sa_status st) {
  if (st == SA_OK && c->trace) {
    collect_trace(c);
  } else {
    // Events of a failed build may not have completed.
    c->recs.clear();
    c->event_used = 0;
  }
}

sa_status build_impl(sa_ctx* c, const u8* text, u64 n, u32 max_rounds, u32* d_sa, u32* d_isa,
                     hipStream_t s) {
  if (!c) return SA_EINVAL;
  sa_status st = build_rounds(c, text, n, max_rounds, d_sa, d_isa, s);
  settle_trace(c, st);
  return st;
}

// Carves the control block (histograms, tickets, counters, plan, alphabet
// tables, lazy-ISA sample) out of kSmallBytes at p.
void bind_small(sa_ctx* c, char* p) {
  c->hist_in = reinterpret_cast<u32*>(p);
  c->hist_run = c->hist_in + kChunkHistWords;
  c->tickets = c->hist_run + kChunkHistWords;
  p += kSmallHist;
  c->counters = reinterpret_cast<u64*>(p);
  c->rc = reinterpret_cast<RoundCtl*>(p + kSmallCounters);
  c->plan_log = reinterpret_cast<u32*>(p + kSmallCounters + kSmallRoundCtl);
  p += kMirrorBytes;
  c->ctl = reinterpret_cast<SortCtl*>(p);
  p += kSmallCtl;
  c->plan = reinterpret_cast<SortPlan*>(p);
  p += kSmallPlan;
  c->present = reinterpret_cast<u32*>(p);
  p += kSmallPresent;
  c->code = reinterpret_cast<u16*>(p);
  p += kSmallCode;
  c->sample = reinterpret_cast<u64*>(p);
  p += kSmallSample;
  c->stage_hist = reinterpret_cast<u32*>(p);
}

// ---------------------------------------------------------------------------
// Workspace of sa_build_noalloc: a file-scope device array holding everything a
// build of up to SA_NOALLOC_MAX_N suffixes needs, so that the call allocates
// nothing. Each GPU holds its own copy from the library's load until the
// process ends. In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress, once per device.
constexpr u64 kNoAllocCap = SA_NOALLOC_MAX_N;

struct ScratchLayout {
  size_t keysA, keysB, valsA, valsB, isa, act_idx, act_rank, live, status, small, bytes;
};

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

constexpr ScratchLayout scratch_layout() {
  ScratchLayout L{};
  size_t at = 0;
  L.keysA = at, at += align256(kNoAllocCap * 8);
  L.keysB = at, at += align256(kNoAllocCap * 8);
  L.valsA = at, at += align256(kNoAllocCap * 4);
  L.valsB = at, at += align256(kNoAllocCap * 4);
  L.isa = at, at += align256(kNoAllocCap * 4);
  L.act_idx = at, at += align256(kNoAllocCap * 4);
  L.act_rank = at, at += align256(kNoAllocCap * 4);
  L.live = at, at += align256((kNoAllocCap + 31) / 32 * 4);
  L.status = at, at += align256(((kNoAllocCap + kSortTileMin - 1) / kSortTileMin + 1) * kRadix * 8);
  L.small = at, at += align256(kSmallBytes);
  L.bytes = at;
  return L;
}
constexpr ScratchLayout kScratch = scratch_layout();
static_assert(kScratch.act_rank == kScratch.act_idx + kNoAllocCap * 4,
              "the active list's ranks follow its positions (one u64 array in quadrupling rounds)");

static __device__ __align__(256) unsigned char scratch[kScratch.bytes];

// Per device: the array's device address and the look-back generation of its
// status words (the array is shared by every context on the device).
struct NoAllocDevice {
  unsigned char* ptr = nullptr;
  u32 gen = 0;
};
std::mutex g_noalloc_mu;
std::vector<NoAllocDevice> g_noalloc;

// Called by sa_ctx_create with `device` current: looks the array's address up
// on this device the first time and clears its status words once.
sa_status noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (device < 0) return SA_EINVAL;
  if (size_t(device) >= g_noalloc.size()) g_noalloc.resize(size_t(device) + 1);
  NoAllocDevice& d = g_noalloc[size_t(device)];
  if (d.ptr) return SA_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return SA_EDEVICE;
  }
  unsigned char* base = static_cast<unsigned char*>(p);
  if (hipMemset(base + kScratch.status, 0, sort_status_words(kNoAllocCap) * sizeof(u64)) !=
          hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    return SA_EDEVICE;
  }
  if (init_small(reinterpret_cast<char*>(base + kScratch.small)) != SA_OK) return SA_EDEVICE;
  d.ptr = base;
  d.gen = 1;
  return SA_OK;
}

// Everything a build reads from the context's workspace, swapped out while the
// scratch array stands in for it.
struct WorkspaceView {
  u64 cap;
  u64 *keysA, *keysB;
  u32 *valsA, *valsB, *isa, *live, *act_idx, *act_rank;
  u64* status;
  u32 *hist_in, *hist_run, *tickets;
  u64* counters;
  RoundCtl* rc;
  u32* plan_log;
  SortCtl* ctl;
  SortPlan* plan;
  u32* present;
  u16* code;
  u64* sample;
  u32 gen;
  bool trace;
  bool graphs_blocked;
};

WorkspaceView save_view(const sa_ctx* c) {
  return WorkspaceView{c->cap,      c->keysA,    c->keysB,        c->valsA,    c->valsB,
                       c->isa,      c->live,     c->act_idx,      c->act_rank, c->status,
                       c->hist_in,  c->hist_run, c->tickets,      c->counters, c->rc,
                       c->plan_log, c->ctl,      c->plan,         c->present,  c->code,
                       c->sample,   c->gen,      c->trace,        c->graphs_blocked};
}

void restore_view(sa_ctx* c, const WorkspaceView& v) {
  c->cap = v.cap;
  c->keysA = v.keysA;
  c->keysB = v.keysB;
  c->valsA = v.valsA;
  c->valsB = v.valsB;
  c->isa = v.isa;
  c->live = v.live;
  c->act_idx = v.act_idx;
  c->act_rank = v.act_rank;
  c->status = v.status;
  c->hist_in = v.hist_in;
  c->hist_run = v.hist_run;
  c->tickets = v.tickets;
  c->counters = v.counters;
  c->rc = v.rc;
  c->plan_log = v.plan_log;
  c->ctl = v.ctl;
  c->plan = v.plan;
  c->present = v.present;
  c->code = v.code;
  c->sample = v.sample;
  c->gen = v.gen;
  c->trace = v.trace;
  c->graphs_blocked = v.graphs_blocked;
}

}  // namespace drv

using namespace drv;

extern "C" {

sa_status sa_ctx_create(sa_ctx** out, int device, const char* tune_cache_json) {
  if (!out) return SA_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return ndev == 0 ? SA_EDEVICE : SA_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) return SA_EDEVICE;
  sa_ctx* c = new (std::nothrow) sa_ctx();
  if (!c) return SA_ENOMEM;
  c->device = device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0)
    c->num_cus = cus;
  std::memset(c->stats, 0, sizeof(c->stats));
  std::memset(&c->info, 0, sizeof(c->info));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->arch = prop.gcnArchName;
    const size_t colon = c->arch.find(':');
    if (colon != std::string::npos) c->arch.resize(colon);
  }
  if (tune_cache_json && tune_cache_json[0]) {
    c->tune = new (std::nothrow) TuneTable();
    if (!c->tune) {
      delete c;
      return SA_ENOMEM;
    }
    c->tune_path = tune_cache_json;
    const sa_status ts = tune_load(tune_cache_json, *c->tune);
    if (ts != SA_OK) {
      delete c->tune;
      delete c;
      return ts;
    }
  }
  if (hipMalloc(&c->small, kSmallBytes) != hipSuccess) {
    delete c;
    return SA_ENOMEM;
  }
  bind_small(c, static_cast<char*>(c->small));
  if (init_small(static_cast<char*>(c->small)) != SA_OK || noalloc_setup(device) != SA_OK) {
    sa_ctx_destroy(c);
    return SA_EDEVICE;
  }
  if (hipHostMalloc(&c->h_mirror, kMirrorBytes) != hipSuccess) {
    c->h_mirror = nullptr;
    sa_ctx_destroy(c);
    return SA_ENOMEM;
  }
  c->h_counters = static_cast<u64*>(c->h_mirror);
  c->h_rc = reinterpret_cast<RoundCtl*>(static_cast<char*>(c->h_mirror) + kSmallCounters);
  c->h_plans = reinterpret_cast<u32*>(static_cast<char*>(c->h_mirror) + kSmallCounters +
                                      kSmallRoundCtl);
  *out = c;
  return SA_OK;
}

sa_status sa_ctx_destroy(sa_ctx* ctx) {
  if (!ctx) return SA_OK;
  (void)hipSetDevice(ctx->device);
  free_workspace(ctx);
  free_pair_workspace(ctx);
  free_level_bufs(ctx);
  drop_graphs(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  (void)hipFree(ctx->small);
  if (ctx->h_mirror) (void)hipHostFree(ctx->h_mirror);
  (void)hipFree(ctx->toff);
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  delete ctx->tune;
  delete ctx;
  return SA_OK;
}

sa_status sa_build(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma, uint32_t* d_sa,
                   void* stream) {
  if (!ctx) return SA_EINVAL;
  if (sigma == 0 || sigma > 256) return SA_EINVAL;
  ctx->sigma_hint = sigma;
  const sa_status st =
      build_impl(ctx, d_text, n, 0, d_sa, nullptr, static_cast<hipStream_t>(stream));
  ctx->sigma_hint = 0;
  return st;
}

sa_status sa_build_noalloc(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma,
                           uint32_t* d_sa, void* stream) {
  if (!ctx) return SA_EINVAL;
  if (sigma == 0 || sigma > 256) return SA_EINVAL;
  if (n > SA_NOALLOC_MAX_N) return SA_ETOOBIG;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (size_t(ctx->device) < g_noalloc.size()) base = g_noalloc[size_t(ctx->device)].ptr;
  }
  if (!base) return SA_EDEVICE;
  // The build runs on the scratch array in place of the context's workspace:
  // a capacity of SA_NOALLOC_MAX_N means no growth, and tracing (which
  // creates events) is off for the call.
  const WorkspaceView saved = save_view(ctx);
  WorkspaceView v = saved;
  v.cap = kNoAllocCap;
  v.keysA = reinterpret_cast<u64*>(base + kScratch.keysA);
  v.keysB = reinterpret_cast<u64*>(base + kScratch.keysB);
  v.valsA = reinterpret_cast<u32*>(base + kScratch.valsA);
  v.valsB = reinterpret_cast<u32*>(base + kScratch.valsB);
  v.isa = reinterpret_cast<u32*>(base + kScratch.isa);
  v.act_idx = reinterpret_cast<u32*>(base + kScratch.act_idx);
  v.act_rank = reinterpret_cast<u32*>(base + kScratch.act_rank);
  v.live = reinterpret_cast<u32*>(base + kScratch.live);
  v.status = reinterpret_cast<u64*>(base + kScratch.status);
  v.trace = false;
  v.graphs_blocked = true;  // capturing a round would allocate
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    v.gen = g_noalloc[size_t(ctx->device)].gen;
  }
  restore_view(ctx, v);
  bind_small(ctx, reinterpret_cast<char*>(base + kScratch.small));
  ctx->sigma_hint = sigma;
  const sa_status st =
      build_impl(ctx, d_text, n, 0, d_sa, nullptr, static_cast<hipStream_t>(stream));
  ctx->sigma_hint = 0;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    g_noalloc[size_t(ctx->device)].gen = ctx->gen;
  }
  restore_view(ctx, saved);
  return st;
}

sa_status sa_build_rounds(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t max_rounds,
                          uint32_t* d_sa, uint32_t* d_isa, void* stream) {
  return build_impl(ctx, d_text, n, max_rounds, d_sa, d_isa, static_cast<hipStream_t>(stream));
}

sa_status sa_last_build_info(const sa_ctx* ctx, sa_build_info* out) {
  if (!ctx || !out) return SA_EINVAL;
  *out = ctx->info;
  return SA_OK;
}

sa_status sa_radix_sort_pairs(sa_ctx* ctx, uint64_t* d_keys, uint32_t* d_vals, uint64_t count,
                              uint32_t key_bits, void* stream) {
  if (!ctx) return SA_EINVAL;
  if (count == 0) return SA_OK;
  if (!d_keys || !d_vals || key_bits == 0 || key_bits > 64) return SA_EINVAL;
  if (count >= (u64(1) << 32)) return SA_ETOOBIG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipSetDevice(ctx->device) != hipSuccess) return SA_EDEVICE;
  sa_status st = ensure_workspace(ctx, count);
  if (st != SA_OK) return st;
  {
    Tracer t(ctx, s, SA_KERNEL_OTHER, 0);
    launch_fill_u64(ctx->counters, kCtrCount, 0, s);
  }
  if (hipMemcpyAsync(ctx->keysA, d_keys, count * sizeof(u64), hipMemcpyDeviceToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(ctx->valsA, d_vals, count * sizeof(u32), hipMemcpyDeviceToDevice, s) !=
          hipSuccess)
    return SA_EDEVICE;
  const int npass = npass_for(ctx, int(key_bits));
  run_sort(ctx, full_bufs(ctx), count, npass, 1, 0, s);
  st = readback(ctx, s);  // also waits for the plan flags
  if (st != SA_OK) {
    ctx->recs.clear();
    ctx->event_used = 0;
    return st;
  }
  const u32 final_buf = ctx->h_plans[3 * kMaxPasses];
  const u64* ksrc = final_buf ? ctx->keysB : ctx->keysA;
  const u32* vsrc = final_buf ? ctx->valsB : ctx->valsA;
  if (hipMemcpyAsync(d_keys, ksrc, count * sizeof(u64), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(d_vals, vsrc, count * sizeof(u32), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SA_EDEVICE;
  if (ctx->trace) collect_trace(ctx);
  return SA_OK;
}

size_t sa_workspace_bytes(uint64_t total_n, uint32_t num_texts) {
  const u64 cap = std::max<u64>(total_n, 1 << 16);
  // keys A/B (u64), values A/B, ISA, active positions and ranks (u32), the
  // live-position bitmap, the sort look-back statuses and the control block.
  u64 bytes = cap * (2 * 8 + 5 * 4) + ceil_div(cap, 32) * 4 + sort_status_words(cap) * 8 +
              kSmallBytes;
  if (num_texts > 1) {
    // A batch also keeps its survivors as (text << 32 | position) and one
    // table row per text.
    bytes += cap * 8 + table_layout(num_texts).bytes;
  }
  return size_t(bytes);
}

sa_status sa_ctx_set_trace(sa_ctx* ctx, int on) {
  if (!ctx) return SA_EINVAL;
  ctx->trace = on != 0;
  return SA_OK;
}

sa_status sa_ctx_set_isa_mode(sa_ctx* ctx, int mode) {
  if (!ctx || mode < SA_ISA_AUTO || mode > SA_ISA_LAZY) return SA_EINVAL;
  ctx->isa_mode = mode;
  return SA_OK;
}

sa_status sa_ctx_set_tuning(sa_ctx* ctx, const sa_tuning* t) {
  if (!ctx) return SA_EINVAL;
  if (!t) {
    ctx->tuning_explicit = false;
    apply_tuning(ctx, default_tuning());
    return SA_OK;
  }
  if (!tuning_valid(*t)) return SA_EINVAL;
  ctx->tuning_explicit = true;
  ctx->explicit_tuning = *t;
  apply_tuning(ctx, *t);
  return SA_OK;
}

sa_status sa_ctx_get_tuning(const sa_ctx* ctx, sa_tuning* out) {
  if (!ctx || !out) return SA_EINVAL;
  *out = current_tuning(ctx);
  return SA_OK;
}

sa_status sa_ctx_tuning_source(const sa_ctx* ctx, int* source) {
  if (!ctx || !source) return SA_EINVAL;
  *source = ctx->tuning_explicit ? 2 : ctx->tuned_from_cache ? 1 : 0;
  return SA_OK;
}

sa_status sa_ctx_reset_stats(sa_ctx* ctx) {
  if (!ctx) return SA_EINVAL;
  std::memset(ctx->stats, 0, sizeof(ctx->stats));
  return SA_OK;
}

sa_status sa_ctx_get_kernel_stats(const sa_ctx* ctx, int kind, sa_kernel_stats* out) {
  if (!ctx || !out || kind < 0 || kind >= SA_KERNEL_KINDS) return SA_EINVAL;
  *out = ctx->stats[kind];
  return SA_OK;
}

const char* sa_strerror(sa_status s) {
  switch (s) {
    case SA_OK: return "ok";
    case SA_EINVAL: return "invalid argument";
    case SA_ENOMEM: return "out of device memory";
    case SA_ETOOBIG: return "input too large (n must be < 2^32 and within the entry point's maximum)";
    case SA_EDEVICE: return "device error";
    case SA_EBUSY: return "busy";
  }
  return "unknown status";
}

}  // extern "C"
