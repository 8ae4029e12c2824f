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

u64 sort_status_words(u64 cap) { return ceil_div(cap, kSortTileMin) * kRadix; }

int bits_of(u64 v) { return v == 0 ? 0 : 64 - __builtin_clzll(v); }

void free_workspace(sa_ctx* c) {
  (void)hipFree(c->keysA);
  (void)hipFree(c->keysB);
  (void)hipFree(c->valsA);
  (void)hipFree(c->valsB);
  (void)hipFree(c->isa);
  (void)hipFree(c->live);
  (void)hipFree(c->act_idx);
  (void)hipFree(c->act_rank);
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
            dev_alloc(&c->valsB, cap) && dev_alloc(&c->isa, cap) && dev_alloc(&c->act_idx, cap) &&
            dev_alloc(&c->live, ceil_div(cap, 32)) &&
            dev_alloc(&c->act_rank, cap) && dev_alloc(&c->status, sort_status_words(cap));
  if (!ok) {
    free_workspace(c);
    return SA_ENOMEM;
  }
  // The status array starts cleared; generations then keep it valid without
  // further clearing.
  if (hipMemset(c->status, 0, sort_status_words(cap) * sizeof(u64)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    free_workspace(c);
    return SA_EDEVICE;
  }
  c->cap = cap;
  c->gen = 0;
  return SA_OK;
}

// Next look-back generation; clears the status array when the 22-bit counter
// wraps.
u32 next_gen(sa_ctx* c, hipStream_t s) {
  if (c->gen + 1 >= kGenMask) {
    launch_fill_u64(c->status, sort_status_words(c->cap), 0, s);
    c->gen = 0;
  }
  return ++c->gen;
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

// Sweep geometry: tiles of block * items pairs, chunks of a power-of-two
// number of tiles so that at most kChunks chunks cover the input.
SortGeom make_geom(u64 count, int items, int block) {
  SortGeom g;
  g.count = count;
  g.tile = u32(block * items);
  const u64 tiles = std::max<u64>(1, ceil_div(count, g.tile));
  const u64 per = ceil_div(tiles, kChunks);
  u32 lg = 0;
  while ((u64(1) << lg) < per) ++lg;
  g.ct_log2 = lg;
  g.nchunks = u32(ceil_div(tiles, u64(1) << lg));
  return g;
}

// Sweep workgroups one CU holds at once for each tile shape (register and LDS
// limits of the kernel instances).
int default_wgs_per_cu(int items, int block, bool table) {
  // The runtime's occupancy figure for the shape, cached per shape; if the
  // query fails, what one CU's 160 KB of LDS holds: the key tile, the per-wave
  // digit counts (16 bits), the 16-bit chunk histograms of the next sweep, the
  // match table if any and about 4 KB of small arrays.
  static std::atomic<int> cache[2][2][32];
  const int bi = block == 2 * kRadix ? 1 : 0;
  const int ii = items & 31;
  const int ti = table ? 1 : 0;
  int n = cache[ti][bi][ii].load(std::memory_order_relaxed);
  if (n > 0) return n;
  n = onesweep_wgs_per_cu(items, block, table);
  if (n <= 0) {
    const int lds = block * items * 8 + (block / kWave / 2) * kRadix * 4 + kChunks * kRadix * 2 +
                    (table ? (block / kWave) * kRadix * 8 : 0) + 4096;
    n = (160 * 1024) / lds;
    if (n < 1) n = 1;
    return n;
  }
  cache[ti][bi][ii].store(n, std::memory_order_relaxed);
  return n;
}

// Sorts (kA, vA or generated values) by the low 8*npass bits. The sorted pairs
// end in the buffer named by plan->final_buf. The plan flags are copied to
// h_plans slot `slot` on the stream.
void run_sort(sa_ctx* c, const Bufs& bf, u64 count, int npass, int vals_present, int slot,
              hipStream_t s) {
  const SortGeom geo = make_geom(count, c->sort_items, c->sort_block);
  const bool table = c->sort_match == 1;
  {
    Tracer t(c, s, SA_KERNEL_OTHER, 0);
    // Chunk histograms and tickets; tile tickets, the key ORs and the
    // survivor count the re-rank adds to.
    static_assert(kCtrSortTiles < kCtrActive && kCtrKeyOr < kCtrActive && kCtrKeyNot < kCtrActive,
                  "one fill clears the sort's counters");
    launch_fill_u32(c->hist_in, 2 * kChunkHistWords + kTicketWords, 0, s);
    launch_fill_u64(c->counters, kCtrActive + 1, 0, s);
  }
  {
    Tracer t(c, s, SA_KERNEL_HISTOGRAM, double(count) * 8.0);
    launch_radix_histogram(bf.kA, geo, c->hist_in, c->counters, s);
  }
  {
    Tracer t(c, s, SA_KERNEL_OTHER, 0);
    launch_radix_plan(c->counters, npass, vals_present, c->plan, s);
    launch_radix_histogram_first(bf.kA, geo, c->plan, c->hist_in, s);
  }
  (void)hipMemcpyAsync(c->h_plans + size_t(slot) * kPlanFlagWords, c->plan->skip,
                       kPlanFlagWords * sizeof(u32), hipMemcpyDeviceToHost, s);
  const u64 tiles = ceil_div(count, geo.tile);
  const int per_cu = c->sort_wgs_per_cu > 0
                         ? c->sort_wgs_per_cu
                         : default_wgs_per_cu(c->sort_items, c->sort_block, table);
  const u64 want = std::min<u64>(tiles, u64(c->num_cus) * u64(per_cu));
  const u32 grid = u32(std::max<u64>(1, want / geo.nchunks) * geo.nchunks);
  for (int p = 0; p < npass; ++p) {
    u32 gen = next_gen(c, s);
    Tracer t(c, s, SA_KERNEL_SORT_PASS, 0, slot, p, count);
    launch_onesweep_pass(bf.kA, bf.kB, bf.vA, bf.vB, geo, p, c->plan, c->hist_in, c->hist_run,
                         c->tickets, c->status, c->counters, gen, c->sort_items,
                         c->sort_block, table, grid, s);
  }
}

void run_rerank(sa_ctx* c, const Bufs& bf, const RerankArgs& args, u32* d_sa, hipStream_t s) {
  const double count = double(args.count);
  // 12 bytes read per element; 4 written (ISA, SA or survivor name) plus 4 for a
  // survivor's position, counted as 4 per element either way.
  double bytes = count * 16.0 - ((args.mode & kRerankScatterIsa) ? 0.0 : 4.0 * count);
  if (args.mode & kRerankIsaOnly) bytes = count * 16.0;
  Tracer t(c, s, (args.mode & kRerankIsaOnly) ? SA_KERNEL_ISA_SCATTER : SA_KERNEL_RERANK, bytes);
  launch_rerank_compact(bf.kA, bf.kB, bf.vA, bf.vB, c->plan, args, c->isa, d_sa,
                        args.tbase ? nullptr : c->act_idx, args.tbase ? c->act_ti : nullptr,
                        c->act_rank, c->counters, s);
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
  if (hipMemcpyAsync(c->h_counters, c->counters, kCtrCount * sizeof(u64), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
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
    launch_fill_u64(reinterpret_cast<u64*>(c->present), 256 / 2, 0, s);
  }
  {
    Tracer t(c, s, SA_KERNEL_OTHER, double(n));
    launch_byte_presence(text, n, c->present, s);
    launch_alphabet_codes(c->present, c->code, c->counters, c->round0_trim, 0, s);
  }
  {
    Tracer t(c, s, SA_KERNEL_PACK_TEXT, double(n) * 9.0);
    launch_pack_text(text, n, c->code, c->counters, c->keysA, s);
  }
  run_sort(c, full, n, kMaxPasses, 0, 0, s);
  run_rerank(c, full, single_args(n, n, 0, 0), d_sa, s);
  st = readback(c, s);
  if (st != SA_OK) return st;

  sa_build_info& info = c->info;
  info.sigma = u32(c->h_counters[kCtrSigma]);
  info.code_bits = u32(c->h_counters[kCtrCodeBits]);
  info.chars0 = u32(c->h_counters[kCtrChars]);
  info.rounds = 1;
  info.active[0] = n;
  info.key_bits[0] = info.code_bits * info.chars0;
  info.passes_run[0] = passes_run(c, 0, kMaxPasses);
  u64 h = info.chars0;
  info.prefix_len = h;
  u64 active = c->h_counters[kCtrActive];

  // ISA after round 0: eager scatter, or lazy (survivors only) when few
  // suffixes survive and the later rounds' buffers fit in the spare keys.
  const u32 f0 = final_buf_of(c, 0);
  const u64* keys0 = f0 ? c->keysB : c->keysA;
  u64* spare = f0 ? c->keysA : c->keysB;
  // Later-round buffers are carved at 256-byte boundaries (vector accesses).
  const u64 a1 = (std::max<u64>(active, 1) + 63) / 64 * 64;
  const bool fits = a1 * 24 <= n * 8;
  bool lazy = false;
  if (c->isa_mode == SA_ISA_LAZY)
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
      run_rerank(c, full, single_args(n, n, 0, kRerankScatterIsa | kRerankIsaOnly), d_sa, s);
    }
  }
  // Later rounds sort at most `active` pairs; in lazy mode their buffers are
  // carved out of the spare keys so that the round-0 sorted keys stay intact.
  Bufs later = full;
  if (lazy) {
    later.kA = spare;
    later.kB = spare + a1;
    later.vA = reinterpret_cast<u32*>(spare + 2 * a1);
    later.vB = later.vA + a1;
  }

  // Later rounds: only suffixes whose name is still shared.
  const int b = bits_of(n);  // ranks and second ranks are <= n
  const int key_bits = 2 * b;
  const int npass = int(ceil_div(u64(key_bits), kRadixBits));
  while (active > 0 && (max_rounds == 0 || info.rounds < max_rounds)) {
    if (info.rounds >= SA_MAX_ROUNDS) return SA_EDEVICE;  // cannot happen for n < 2^32
    const int slot = int(info.rounds);
    {
      Tracer t(c, s, SA_KERNEL_PACK_PAIRS, double(active) * 24.0);
      if (lazy)
        launch_pack_pairs_lazy(c->act_idx, c->act_rank, active, n, h, b, c->isa, text, c->code,
                               c->counters, keys0, c->sample, c->live, later.kA, later.vA, s);
      else
        launch_pack_pairs(c->act_idx, c->act_rank, active, n, h, b, c->isa, later.kA, later.vA,
                          s);
    }
    run_sort(c, later, active, npass, 1, slot, s);
    run_rerank(c, later, single_args(active, n, b, kRerankScatterIsa), d_sa, s);
    st = readback(c, s);
    if (st != SA_OK) return st;
    info.active[slot] = active;
    info.key_bits[slot] = u32(key_bits);
    info.passes_run[slot] = passes_run(c, slot, npass);
    info.rounds += 1;
    h *= 2;
    info.prefix_len = h;
    active = c->h_counters[kCtrActive];
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
  c->counters = reinterpret_cast<u64*>(p + kSmallHist);
  c->plan = reinterpret_cast<SortPlan*>(p + kSmallHist + kSmallCounters);
  c->present = reinterpret_cast<u32*>(p + kSmallHist + kSmallCounters + kSmallPlan);
  c->code = reinterpret_cast<u16*>(p + kSmallHist + kSmallCounters + kSmallPlan + kSmallPresent);
  c->sample = reinterpret_cast<u64*>(p + kSmallHist + kSmallCounters + kSmallPlan + kSmallPresent +
                                     kSmallCode);
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
  L.status = at, at += align256((kNoAllocCap + kSortTileMin - 1) / kSortTileMin * kRadix * 8);
  L.small = at, at += align256(kSmallBytes);
  L.bytes = at;
  return L;
}
constexpr ScratchLayout kScratch = scratch_layout();

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
  d.ptr = base;
  d.gen = 0;
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
  SortPlan* plan;
  u32* present;
  u16* code;
  u64* sample;
  u32 gen;
  bool trace;
};

WorkspaceView save_view(const sa_ctx* c) {
  return WorkspaceView{c->cap,      c->keysA,   c->keysB,    c->valsA,    c->valsB,
                       c->isa,      c->live,    c->act_idx,  c->act_rank, c->status,
                       c->hist_in,  c->hist_run, c->tickets, c->counters, c->plan,
                       c->present,  c->code,    c->sample,   c->gen,      c->trace};
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
  c->plan = v.plan;
  c->present = v.present;
  c->code = v.code;
  c->sample = v.sample;
  c->gen = v.gen;
  c->trace = v.trace;
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
  if (noalloc_setup(device) != SA_OK) {
    sa_ctx_destroy(c);
    return SA_EDEVICE;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_counters), kCtrCount * sizeof(u64)) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_plans),
                    size_t(SA_MAX_ROUNDS + 1) * kPlanFlagWords * sizeof(u32)) != hipSuccess) {
    sa_ctx_destroy(c);
    return SA_ENOMEM;
  }
  *out = c;
  return SA_OK;
}

sa_status sa_ctx_destroy(sa_ctx* ctx) {
  if (!ctx) return SA_OK;
  (void)hipSetDevice(ctx->device);
  free_workspace(ctx);
  (void)hipFree(ctx->small);
  if (ctx->h_counters) (void)hipHostFree(ctx->h_counters);
  if (ctx->h_plans) (void)hipHostFree(ctx->h_plans);
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
  const int npass = int(ceil_div(key_bits, kRadixBits));
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
