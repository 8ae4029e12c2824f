// Multi-text engine: batched builds (sa_build_batch) and the continuous-
// batching server (sa_server_*).
//
// Prefix doubling with discarding (Section 2.1, Alg. 5) for many texts at once.
// Every text has a slot; keys carry the slot in their top bits, so one sort and
// one re-rank per round serve all texts while names stay per text. A text's
// first round packs its own alphabet's codes (round-0 keys); later rounds pair
// its rank with the rank h_t positions on. Texts may join at any round: a
// round merges texts at round 0 with texts at later rounds, because keys of
// different texts are never compared beyond their slot bits.

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "driver.h"

using namespace drv;

namespace {

}  // namespace

namespace drv {

// Byte offsets of the per-slot device tables in the engine's one allocation.
// The tables written by the host each round come first, contiguous, so that
// one copy from a pinned mirror uploads them all.
TableLayout table_layout(u32 nslots) {
  TableLayout L{};
  const size_t S = nslots;
  size_t bytes = 0;
  auto take = [&](size_t b) {
    const size_t at = bytes;
    bytes += (b + 255) / 256 * 256;
    return at;
  };
  L.o_base = take(S * 8);
  L.o_len = take(S * 8);
  L.o_h = take(S * 8);
  L.o_start = take(S * 8);
  L.o_r0 = take(S);
  L.o_nt = take(S * 4);
  L.o_no = take((S + 1) * 8);
  L.o_nc = take((S + 1) * 8);
  L.up_bytes = bytes;
  L.o_code = take(S * 256 * 2);
  L.o_pres = take(S * 32);
  L.o_wc = take(S * 4);
  L.o_surv = take(S * 4);
  L.bytes = bytes;
  return L;
}

}  // namespace drv

namespace {

// Device tables and host mirrors of the text slots.
struct Engine {
  sa_ctx* c = nullptr;
  u32 slots = 0;
  int idbits = 0;   // slot bits at the top of every later-round key
  int B = 0;        // bits of a rank
  // Where the slot sits in round-0 keys: 64 - idbits (the top, as in later
  // rounds, whose keys a round-0 text shares its sort with), or lower, right
  // above the characters, when every text starts round 0 together.
  int round0_shift = 0;
  void* dev = nullptr;  // one allocation for all tables
  TextTab tab{};
  u32* d_new_t = nullptr;
  u64* d_new_out = nullptr;
  u64* d_new_chunk0 = nullptr;
  // host mirrors
  std::vector<u64> base, len, h;
  std::vector<u32> chars, round;
  std::vector<u8> busy, round0;
  u32* h_wc = nullptr;    // pinned
  u32* h_surv = nullptr;  // pinned
  char* h_up = nullptr;   // pinned mirror of the per-round upload tables
  size_t up_bytes = 0, o_up_base = 0, o_up_len = 0, o_up_h = 0, o_up_start = 0, o_up_r0 = 0,
         o_up_nt = 0, o_up_no = 0, o_up_nc = 0;
  std::vector<u64> start;  // host mirror of tab.start
  u64 active = 0;         // survivors carried into the next round
  std::vector<u32> live;  // slots with elements in the active set or joining now
  // Batched build only (every text starts round 0 together): round 0 writes no
  // ISA; it is then formed eagerly (an ISA-only second pass of the round-0
  // re-rank) or, when few suffixes survive, lazily.
  bool defer_round0_isa = false;
  bool lazy = false;           // the ISA holds the survivors' names only (live bitmap)
  const u64* keys0 = nullptr;  // lazy: round-0 sorted keys
  Bufs later{};                // lazy: later rounds' buffers, carved from the spare keys
  RerankArgs last_args{};      // the last round's re-rank

  ~Engine() { release(); }
  void release() {
    (void)hipFree(dev);
    dev = nullptr;
    if (h_wc) (void)hipHostFree(h_wc);
    if (h_surv) (void)hipHostFree(h_surv);
    if (h_up) (void)hipHostFree(h_up);
    h_wc = h_surv = nullptr;
    h_up = nullptr;
  }

  sa_status init(sa_ctx* ctx, u32 nslots, int id_bits, int rank_bits) {
    c = ctx;
    slots = nslots;
    idbits = id_bits;
    B = rank_bits;
    round0_shift = 64 - id_bits;
    const TableLayout L = table_layout(nslots);
    const size_t S = nslots;
    const size_t bytes = L.bytes;
    const size_t o_base = L.o_base, o_len = L.o_len, o_h = L.o_h, o_r0 = L.o_r0, o_nt = L.o_nt,
                 o_no = L.o_no, o_nc = L.o_nc, o_code = L.o_code, o_pres = L.o_pres,
                 o_wc = L.o_wc, o_surv = L.o_surv;
    up_bytes = L.up_bytes;
    o_up_base = o_base, o_up_len = o_len, o_up_h = o_h, o_up_r0 = o_r0, o_up_nt = o_nt,
    o_up_no = o_no, o_up_nc = o_nc;
    o_up_start = L.o_start;
    if (hipMalloc(&dev, bytes) != hipSuccess) {
      dev = nullptr;
      (void)hipGetLastError();
      return SA_ENOMEM;
    }
    if (hipMemset(dev, 0, bytes) != hipSuccess) return SA_EDEVICE;
    char* p = static_cast<char*>(dev);
    tab.base = reinterpret_cast<u64*>(p + o_base);
    tab.len = reinterpret_cast<u64*>(p + o_len);
    tab.code = reinterpret_cast<u16*>(p + o_code);
    tab.present = reinterpret_cast<u32*>(p + o_pres);
    tab.wc = reinterpret_cast<u32*>(p + o_wc);
    tab.h = reinterpret_cast<u64*>(p + o_h);
    tab.round0 = reinterpret_cast<u8*>(p + o_r0);
    tab.surv = reinterpret_cast<u32*>(p + o_surv);
    tab.start = reinterpret_cast<u64*>(p + L.o_start);
    d_new_t = reinterpret_cast<u32*>(p + o_nt);
    d_new_out = reinterpret_cast<u64*>(p + o_no);
    d_new_chunk0 = reinterpret_cast<u64*>(p + o_nc);
    if (hipHostMalloc(reinterpret_cast<void**>(&h_wc), S * 4) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h_surv), S * 4) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h_up), up_bytes) != hipSuccess)
      return SA_ENOMEM;
    base.assign(S, 0);
    start.assign(S, 0);
    len.assign(S, 0);
    h.assign(S, 0);
    chars.assign(S, 0);
    round.assign(S, 0);
    busy.assign(S, 0);
    round0.assign(S, 0);
    active = 0;
    live.clear();
    return SA_OK;
  }

  // One merged round: the texts in `joining` (slots whose base/len are set)
  // start round 0; every text with survivors does its next round. Fills
  // `finished` with the slots whose suffixes are all final. SA entries go to
  // sa_arena[base + rank - 1], names to c->isa[base + i].
  sa_status round_step(const u8* text_arena, u32* sa_arena, const std::vector<u32>& joining,
                       std::vector<u32>& finished, int slot_info, hipStream_t s) {
    finished.clear();
    // A lazy ISA holds only the survivors' names and the round-0 sorted keys
    // of the texts already running; a text joining now would overwrite those
    // keys. Refused before anything is enqueued.
    if (lazy) {
      for (u32 t : joining)
        if (len[t] != 0) return SA_EINVAL;
    }
    const Bufs full = full_bufs(c);
    const int idshift = 64 - idbits;
    // Round-0 keys below the top share no sort with later-round keys.
    const bool compact0 = round0_shift != idshift;
    if (compact0 && !live.empty() && !joining.empty()) return SA_EINVAL;
    // Work list of the joining texts.
    std::vector<u32> nt;
    std::vector<u64> nout(1, 0), nchunk(1, 0);
    for (u32 t : joining) {
      if (len[t] == 0) {
        finished.push_back(t);
        continue;
      }
      nt.push_back(t);
      nout.push_back(nout.back() + len[t]);
      nchunk.push_back(nchunk.back() + ceil_div(len[t], kNewChunk));
    }
    const u32 m = u32(nt.size());
    const u64 A0 = nout.back();
    // Per-slot table updates: joining texts get base/len/round0; texts that
    // finished round 0 last time switch to pair keys with their own h.
    for (u32 t : live) {
      if (round0[t]) round0[t] = 0;
      h[t] = u64(chars[t]) << (round[t] - 1);
    }
    for (u32 t : nt) round0[t] = 1;
    // The sorted array holds each text's elements together, in slot order:
    // the joining texts' whole length, the others' survivors of last round.
    std::fill(start.begin(), start.end(), u64(0));
    {
      std::vector<u64> cnt(slots, 0);
      for (u32 t : nt) cnt[t] = len[t];
      for (u32 t : live) cnt[t] = h_surv[t];
      u64 at = 0;
      for (u32 t = 0; t < slots; ++t) {
        start[t] = at;
        at += cnt[t];
      }
    }
    // Upload the per-round tables (a few values per slot) in one copy from
    // the pinned mirror. The previous round synchronised the stream, so the
    // mirror is free to be rewritten.
    std::memcpy(h_up + o_up_base, base.data(), slots * 8);
    std::memcpy(h_up + o_up_len, len.data(), slots * 8);
    std::memcpy(h_up + o_up_h, h.data(), slots * 8);
    std::memcpy(h_up + o_up_start, start.data(), slots * 8);
    std::memcpy(h_up + o_up_r0, round0.data(), slots);
    if (m) {
      std::memcpy(h_up + o_up_nt, nt.data(), m * 4);
      std::memcpy(h_up + o_up_no, nout.data(), (m + 1) * 8);
      std::memcpy(h_up + o_up_nc, nchunk.data(), (m + 1) * 8);
    }
    const size_t up = m ? o_up_nc + (m + 1) * 8 : o_up_r0 + slots;
    if (hipMemcpyAsync(dev, h_up, up, hipMemcpyHostToDevice, s) != hipSuccess)
      return SA_EDEVICE;
    NewList nl{d_new_t, d_new_out, d_new_chunk0, m, nchunk.back()};
    {
      Tracer tr(c, s, SA_KERNEL_OTHER, 0);
      launch_fill_u64(c->counters, kCtrCount, 0, s);
      launch_fill_u32(tab.surv, slots, 0, s);
    }
    if (m) {
      {
        Tracer tr(c, s, SA_KERNEL_OTHER, double(A0));
        launch_multi_presence(text_arena, tab, nl, s);
        // A compact layout's character budget ends on a digit boundary already.
        launch_multi_codes(tab, nl, idbits, round0_shift, compact0 ? 0 : c->round0_trim,
                           c->radix_bits, s);
      }
      Tracer tr(c, s, SA_KERNEL_PACK_TEXT, double(A0) * 13.0);
      launch_multi_pack0(text_arena, tab, nl, round0_shift, c->keysA, c->valsA, s);
    }
    const Bufs bufs = lazy ? later : full;
    if (active) {
      Tracer tr(c, s, SA_KERNEL_PACK_PAIRS, double(active) * 24.0);
      if (lazy)
        launch_multi_pack_pairs_lazy(c->act_ti, c->act_rank, active, tab, B, idshift,
                                     round0_shift, c->isa, c->live, text_arena, keys0, bufs.kA,
                                     bufs.vA, s);
      else
        launch_multi_pack_pairs(c->act_ti, c->act_rank, active, tab, B, idshift, c->isa,
                                c->keysA + A0, c->valsA + A0, s);
    }
    const u64 total = A0 + active;
    if (total) {
      run_sort(c, bufs, total, npass_for(c, 64), 1, slot_info, s);
      RerankArgs a{};
      a.count = total;
      a.n = 0;
      a.gshift = B;  // group = (slot, rank) for texts past round 0
      a.rshift = B;
      a.rmask = (u64(1) << B) - 1;
      a.idshift = m ? round0_shift : idshift;  // (equal when the round mixes)
      a.mode = (defer_round0_isa && m) ? 0 : kRerankScatterIsa;
      a.tbase = tab.base;
      a.tlen = tab.len;
      a.tround0 = tab.round0;
      a.tstart = tab.start;
      run_rerank(c, bufs, a, sa_arena, total, total, s);
      last_args = a;
      // Survivors per text; their number is read on the device.
      Tracer tr(c, s, SA_KERNEL_OTHER, 0);
      launch_multi_count_survivors(c->act_ti, c->counters + kCtrActive, total, tab.surv, s);
    }
    if (hipMemcpyAsync(h_surv, tab.surv, slots * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      return SA_EDEVICE;
    if (m && hipMemcpyAsync(h_wc, tab.wc, slots * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      return SA_EDEVICE;
    sa_status st = readback(c, s);  // synchronises the stream
    if (st != SA_OK) return st;
    const u64 next_active = total ? c->h_counters[kCtrActive] : 0;
    // Advance every text that took part.
    std::vector<u32> next_live;
    auto advance = [&](u32 t) {
      round[t] += 1;
      if (h_surv[t] == 0) {
        finished.push_back(t);
      } else {
        next_live.push_back(t);
      }
    };
    for (u32 t : nt) {
      chars[t] = h_wc[t] >> 16;
      advance(t);
    }
    for (u32 t : live) advance(t);
    live.swap(next_live);
    active = next_active;
    return SA_OK;
  }

  // Batched build, after round 0 (which ran with defer_round0_isa): forms the
  // ISA eagerly (every name), or lazily (survivors only) when at most
  // 1/lazy_ratio of the n suffixes survive and the later rounds' buffers fit in
  // the spare keys (the context's ISA mode may force either form).
  sa_status form_isa_after_round0(u64 n, hipStream_t s) {
    const u32 f0 = final_buf_of(c, 0);
    const u64* k0 = f0 ? c->keysB : c->keysA;
    u64* spare = f0 ? c->keysA : c->keysB;
    const u64 a1 = (std::max<u64>(active, 1) + 63) / 64 * 64;
    const bool fits = a1 * 24 <= n * 8;
    if (c->isa_mode == SA_ISA_LAZY)
      lazy = active > 0 && fits;
    else if (c->isa_mode == SA_ISA_AUTO)
      lazy = active > 0 && fits && active * c->lazy_ratio <= n;
    else
      lazy = false;
    if (lazy) {
      Tracer t(c, s, SA_KERNEL_OTHER, double(n) / 8.0 + double(active) * 16.0);
      launch_fill_u32(c->live, ceil_div(n, 32), 0, s);
      launch_multi_isa_scatter_list(c->act_ti, c->act_rank, c->counters + kCtrActive, active,
                                    tab, c->isa, c->live, s);
      keys0 = k0;
      later.kA = spare;
      later.kB = spare + a1;
      later.vA = reinterpret_cast<u32*>(spare + 2 * a1);
      later.vB = later.vA + a1;
    } else if (active > 0) {
      // The round-0 re-rank again (same sorted pairs, same per-text tables),
      // writing only the ISA.
      RerankArgs a = last_args;
      a.mode = kRerankScatterIsa | kRerankIsaOnly;
      run_rerank(c, full_bufs(c), a, nullptr, a.count, a.count, s);
    }
    return SA_OK;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// Batched build.

struct sa_batch_state {
  Engine eng;
};

namespace drv {

sa_status build_batch_impl(sa_ctx* c, const u8* text, const u64* h_off, u32 T, u32* d_sa,
                           hipStream_t s) {
  std::memset(&c->info, 0, sizeof(c->info));
  if (!h_off || T == 0) return SA_EINVAL;
  if (h_off[0] != 0) return SA_EINVAL;
  u64 max_n = 0;
  for (u32 t = 0; t < T; ++t) {
    if (h_off[t + 1] < h_off[t]) return SA_EINVAL;
    max_n = std::max<u64>(max_n, h_off[t + 1] - h_off[t]);
  }
  const u64 N = h_off[T];
  c->info.n = N;
  if (max_n >= (u64(1) << 32)) return SA_ETOOBIG;
  // The radix sweep forms output chunk indices in 32 bits from positions
  // shifted right by at least 10 bits; no batch that fits in memory comes near.
  if (N >= (u64(1) << 40)) return SA_ETOOBIG;
  if (N == 0) return SA_OK;
  if (!text || !d_sa) return SA_EINVAL;
  if (T == 1) return build_rounds(c, text, N, 0, d_sa, nullptr, s);
  const int idbits = bits_of(u64(T) - 1);
  const int B = bits_of(max_n);
  if (idbits + 2 * B > 64) return SA_ETOOBIG;
  if (hipSetDevice(c->device) != hipSuccess) return SA_EDEVICE;
  resolve_tuning(c, "batch", N, 0);
  sa_status st = ensure_workspace(c, N);
  if (st != SA_OK) return st;
  if (c->act_ti_cap < c->cap) {
    (void)hipFree(c->act_ti);
    c->act_ti = nullptr;
    c->act_ti_cap = 0;
    if (!dev_alloc(&c->act_ti, c->cap)) return SA_ENOMEM;
    c->act_ti_cap = c->cap;
  }
  Engine eng;
  st = eng.init(c, T, idbits, B);
  if (st != SA_OK) return st;
  eng.defer_round0_isa = true;
  // Every text starts round 0 together, so the round-0 keys need not share
  // the later rounds' layout: the slot goes right above the characters, whose
  // budget (with round0_trim) ends one radix digit below 64 bits, and the
  // first sort runs one sweep fewer than with the slot at the top.
  if (c->round0_trim) {
    const int rb = c->radix_bits;
    const int s0 = (passes_for(64, rb) - 1) * rb - idbits;
    if (s0 >= 9 && s0 < 64 - idbits) eng.round0_shift = s0;  // (a code has at most 9 bits)
  }
  std::vector<u32> joining;
  for (u32 t = 0; t < T; ++t) {
    eng.base[t] = h_off[t];
    eng.len[t] = h_off[t + 1] - h_off[t];
    joining.push_back(t);
  }
  std::vector<u32> finished;
  sa_build_info& info = c->info;
  info.n = N;
  u64 in_round = N;
  for (int r = 0;; ++r) {
    if (r >= SA_MAX_ROUNDS) return SA_EDEVICE;
    st = eng.round_step(text, d_sa, r == 0 ? joining : std::vector<u32>(), finished, r, s);
    if (st != SA_OK) return st;
    info.active[r] = in_round;
    info.passes_run[r] = passes_run(c, r, npass_for(c, 64));
    info.key_bits[r] = 64;
    info.rounds = u32(r + 1);
    in_round = eng.active;
    if (r == 0) {
      st = eng.form_isa_after_round0(N, s);
      if (st != SA_OK) return st;
      eng.defer_round0_isa = false;
      info.lazy_isa = eng.lazy ? 1u : 0u;
    }
    if (eng.active == 0) break;
  }
  u32 maxc = 0;
  for (u32 t = 0; t < T; ++t) maxc = std::max(maxc, eng.chars[t]);
  info.chars0 = maxc;
  info.prefix_len = u64(maxc) << (info.rounds - 1);
  return SA_OK;
}

}  // namespace drv

extern "C" sa_status sa_build_batch(sa_ctx* ctx, const uint8_t* d_texts,
                                    const uint64_t* h_offsets, uint32_t num_texts,
                                    uint32_t* d_sas, void* stream) {
  if (!ctx) return SA_EINVAL;
  sa_status st = build_batch_impl(ctx, d_texts, h_offsets, num_texts, d_sas,
                                  static_cast<hipStream_t>(stream));
  settle_trace(ctx, st);
  return st;
}

// ---------------------------------------------------------------------------
// Continuous-batching server. A worker thread owns the GPU work: each loop it
// admits queued requests whose text fits in the device arena while a slot is
// free, copies their texts in, runs one merged round for every live request
// (new ones at round 0, the others at their own next round), and retires the
// requests whose suffixes are all final. A finished request's SA stays in the
// arena until the caller polls it.

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  std::vector<u8> text;  // pageable host copy, used when the pinned pool is full
  u8* pinned = nullptr;  // host copy in the lane's pinned pool, or null
  u64 pin_at = 0;
  u64 n = 0;
  double t_arrive = 0, t_admit = 0, t_done = 0;
  int state = 0;  // 0 queued, 1 running, 2 done, 3 failed, 4 being copied out
  u32 slot = 0;
  u64 base = 0;
  sa_status err = SA_OK;
};

}  // namespace

namespace {

// One lane of the server: its own context, stream, engine, device arena and
// worker thread.
struct Lane {
  sa_ctx* ctx = nullptr;
  Engine eng;
  int device = 0;
  u64 arena_cap = 0;  // positions
  u64 max_text = 0;
  u8* d_text = nullptr;
  u32* d_sa = nullptr;
  hipStream_t stream = nullptr;
  std::map<u64, u64> free_ranges;  // start -> length
  // Pinned host pool holding submitted texts until they are on the device, so
  // that each upload is one direct copy instead of a staged pageable one.
  u8* h_pool = nullptr;
  u64 pool_cap = 0;
  std::map<u64, u64> pool_free;
  std::deque<u64> queue;
  std::unordered_map<u64, std::unique_ptr<Request>> reqs;
  std::vector<u32> free_slots;
  std::vector<u64> slot_ticket;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  // statistics
  u64 completed = 0, failed = 0, suffixes = 0, rounds = 0;
  double busy_s = 0;

  // First-fit range allocation over a free list (start -> length).
  static bool range_alloc(std::map<u64, u64>& fr, u64 n, u64* out) {
    for (auto it = fr.begin(); it != fr.end(); ++it) {
      if (it->second >= n) {
        *out = it->first;
        const u64 rest = it->second - n, start = it->first + n;
        fr.erase(it);
        if (rest) fr[start] = rest;
        return true;
      }
    }
    return false;
  }

  static void range_release(std::map<u64, u64>& fr, u64 start, u64 n) {
    if (n == 0) return;
    auto it = fr.emplace(start, n).first;
    auto nx = std::next(it);
    if (nx != fr.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      fr.erase(nx);
    }
    if (it != fr.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        fr.erase(it);
      }
    }
  }

  bool alloc(u64 n, u64* out) { return range_alloc(free_ranges, n, out); }
  void release(u64 start, u64 n) { range_release(free_ranges, start, n); }

  // Pool ranges are rounded to 64 bytes so that uploads start aligned.
  static u64 pool_len(u64 n) { return (n + 63) & ~u64(63); }

  void drop_host_copy(Request* r) {
    if (r->pinned) {
      range_release(pool_free, r->pin_at, pool_len(r->n));
      r->pinned = nullptr;
    }
    std::vector<u8>().swap(r->text);
  }

  void run() {
    (void)hipSetDevice(device);
    std::vector<u32> joining, finished;
    std::vector<Request*> copies;
    for (;;) {
      joining.clear();
      copies.clear();
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stop) return;
          // Admission in arrival order: a request waits until a slot and
          // arena space for its text are free.
          while (!queue.empty() && !free_slots.empty()) {
            Request* r = reqs[queue.front()].get();
            u64 at = 0;
            if (!alloc(r->n, &at)) break;
            const u32 slot = free_slots.back();
            free_slots.pop_back();
            r->slot = slot;
            r->base = at;
            r->state = 1;
            r->t_admit = now_s();
            slot_ticket[slot] = queue.front();
            eng.base[slot] = at;
            eng.len[slot] = r->n;
            eng.round[slot] = 0;
            eng.chars[slot] = 0;
            joining.push_back(slot);
            copies.push_back(r);
            queue.pop_front();
          }
          if (!joining.empty() || !eng.live.empty()) break;
          cv.wait(lk);
        }
      }
      const double t0 = now_s();
      sa_status st = SA_OK;
      // A text that waited in pageable memory moves to the pinned pool first
      // when there is room: a host copy and one direct upload beat the
      // runtime's chunked staging of pageable memory.
      for (Request* r : copies) {
        if (r->pinned || !h_pool) continue;
        bool got;
        {
          std::lock_guard<std::mutex> lk(mu);
          got = range_alloc(pool_free, pool_len(r->n), &r->pin_at);
        }
        if (got) {
          r->pinned = h_pool + r->pin_at;
          std::memcpy(r->pinned, r->text.data(), r->n);
        }
      }
      for (Request* r : copies) {
        const void* src = r->pinned ? static_cast<const void*>(r->pinned)
                                    : static_cast<const void*>(r->text.data());
        if (hipMemcpyAsync(d_text + r->base, src, r->n, hipMemcpyHostToDevice, stream) !=
            hipSuccess)
          st = SA_EDEVICE;
      }
      if (st == SA_OK) st = eng.round_step(d_text, d_sa, joining, finished, 0, stream);
      // The round ends with a synchronisation, so the uploads are complete (or
      // the stream is in error) and the host copies can go.
      if (st != SA_OK) (void)hipStreamSynchronize(stream);
      const double t1 = now_s();
      std::lock_guard<std::mutex> lk(mu);
      for (Request* r : copies) drop_host_copy(r);
      busy_s += t1 - t0;
      rounds += 1;
      if (st != SA_OK) {
        // Fail every running request; their slots and arena space return.
        for (auto& kv : reqs) {
          Request* r = kv.second.get();
          if (r->state == 1) {
            r->state = 3;
            r->err = st;
            release(r->base, r->n);
            free_slots.push_back(r->slot);
            failed += 1;
          }
        }
        eng.live.clear();
        eng.active = 0;
        cv.notify_all();
        continue;
      }
      for (u32 slot : finished) {
        Request* r = reqs[slot_ticket[slot]].get();
        r->state = 2;
        r->t_done = t1;
        free_slots.push_back(slot);
        completed += 1;
        suffixes += r->n;
      }
      cv.notify_all();
    }
  }
};

}  // namespace

namespace {

// Creates a lane serving texts of at most max_text bytes with capacity_bytes of
// device memory.
sa_status lane_create(std::unique_ptr<Lane>& out, int device, u64 capacity_bytes, u64 max_text) {
  out.reset(new (std::nothrow) Lane());
  if (!out) return SA_ENOMEM;
  Lane* L = out.get();
  L->device = device;
  L->max_text = max_text;
  const int B = bits_of(max_text);
  int idbits = 64 - 2 * B;
  if (idbits < 1) return SA_ETOOBIG;
  if (idbits > 10) idbits = 10;  // at most 1024 requests in flight per lane
  sa_status st = sa_ctx_create(&L->ctx, device, nullptr);
  if (st != SA_OK) return st;
  // Per arena position: text 1 + SA 4 + ISA 4 + keys 16 + values 8 + survivors
  // 16 + look-back status ~1.
  const u64 per = 50;
  L->arena_cap = capacity_bytes / per;
  if (L->arena_cap < max_text) return SA_ENOMEM;
  sa_ctx* c = L->ctx;
  st = ensure_workspace(c, L->arena_cap);
  if (st != SA_OK) return st;
  if (!dev_alloc(&c->act_ti, c->cap)) return SA_ENOMEM;
  c->act_ti_cap = c->cap;
  if (!dev_alloc(&L->d_text, L->arena_cap) || !dev_alloc(&L->d_sa, L->arena_cap))
    return SA_ENOMEM;
  const u32 slots = 1u << idbits;
  st = L->eng.init(c, slots, idbits, B);
  if (st != SA_OK) return st;
  if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess)
    return SA_EDEVICE;
  // Pinned pool: twice the text arena, between 16 MiB and 4 GiB. Texts that do
  // not fit wait in pageable memory instead.
  u64 pool = 2 * L->arena_cap;
  if (pool < (u64(16) << 20)) pool = u64(16) << 20;
  if (pool > (u64(4) << 30)) pool = u64(4) << 30;
  if (hipHostMalloc(reinterpret_cast<void**>(&L->h_pool), pool, hipHostMallocDefault) ==
      hipSuccess) {
    L->pool_cap = pool;
    L->pool_free[0] = pool;
  } else {
    L->h_pool = nullptr;
    (void)hipGetLastError();
  }
  L->free_ranges[0] = L->arena_cap;
  L->slot_ticket.assign(slots, 0);
  // Slots are handed out from the highest down (free_slots is used as a
  // stack), so the top bits of the slot field, and with them the highest key
  // bits, take part from the first request on.
  for (u32 k = 0; k < slots; ++k) L->free_slots.push_back(k);
  try {
    L->worker = std::thread([L] { L->run(); });
  } catch (...) {
    return SA_ENOMEM;
  }
  return SA_OK;
}

void lane_destroy(Lane* L) {
  if (!L) return;
  {
    std::lock_guard<std::mutex> lk(L->mu);
    L->stop = true;
  }
  L->cv.notify_all();
  if (L->worker.joinable()) L->worker.join();
  (void)hipSetDevice(L->device);
  if (L->stream) (void)hipStreamDestroy(L->stream);
  (void)hipFree(L->d_text);
  (void)hipFree(L->d_sa);
  if (L->h_pool) (void)hipHostFree(L->h_pool);
  L->eng.release();
  if (L->ctx) sa_ctx_destroy(L->ctx);
}

sa_status lane_submit(Lane* L, u64 ticket, const uint8_t* h_text, uint64_t n) {
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return SA_ENOMEM;
  r->n = n;
  r->t_arrive = now_s();
  if (n) {
    bool got = false;
    {
      std::lock_guard<std::mutex> lk(L->mu);
      got = L->h_pool && Lane::range_alloc(L->pool_free, Lane::pool_len(n), &r->pin_at);
    }
    if (got) {
      r->pinned = L->h_pool + r->pin_at;
      std::memcpy(r->pinned, h_text, n);
    } else {
      try {
        r->text.assign(h_text, h_text + n);
      } catch (...) {
        return SA_ENOMEM;
      }
    }
  }
  std::lock_guard<std::mutex> lk(L->mu);
  if (n == 0) {
    r->state = 2;
    r->t_admit = r->t_done = r->t_arrive;
    L->completed += 1;
  } else {
    L->queue.push_back(ticket);
  }
  L->reqs[ticket] = std::move(r);
  L->cv.notify_all();
  return SA_OK;
}

sa_status lane_poll(Lane* L, uint64_t ticket, uint32_t* h_sa_out, int* done, double* latency_ms,
                    bool* released) {
  *released = false;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(L->mu);
    auto it = L->reqs.find(ticket);
    if (it == L->reqs.end()) return SA_EINVAL;
    r = it->second.get();
    if (r->state == 3) {
      const sa_status e = r->err;
      L->reqs.erase(it);
      *released = true;
      return e;
    }
    if (r->state != 2) return SA_OK;
    if (r->n && !h_sa_out) {
      *done = 2;  // ready: call again with an output buffer
      return SA_OK;
    }
    r->state = 4;
  }
  sa_status st = SA_OK;
  if (r->n) {
    if (hipSetDevice(L->device) != hipSuccess ||
        hipMemcpy(h_sa_out, L->d_sa + r->base, r->n * sizeof(u32), hipMemcpyDefault) !=
            hipSuccess)
      st = SA_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(L->mu);
  if (latency_ms) *latency_ms = (r->t_done - r->t_arrive) * 1e3;
  L->release(r->base, r->n);
  L->reqs.erase(ticket);
  L->cv.notify_all();
  *released = true;
  if (st == SA_OK) *done = 1;
  return st;
}

}  // namespace

// The server: size-class lanes, each a continuous-batching engine on its own
// stream, so that short requests are never queued behind the sort of a long
// text's round.
struct sa_server {
  int device = 0;
  u64 max_text = 0;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::vector<u64> lane_max;  // lane k takes texts with n <= lane_max[k]
  std::mutex mu;
  std::unordered_map<u64, int> owner;
  u64 next_ticket = 1;
};

extern "C" {

sa_status sa_server_create(sa_server** out, int device, uint64_t capacity_bytes,
                           uint64_t max_text) {
  if (!out) return SA_EINVAL;
  *out = nullptr;
  if (max_text == 0) max_text = u64(1) << 26;
  if (max_text >= (u64(1) << 32)) return SA_ETOOBIG;
  if (64 - 2 * bits_of(max_text) < 1) return SA_ETOOBIG;
  if (capacity_bytes == 0) {
    if (hipSetDevice(device) != hipSuccess) return SA_EDEVICE;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return SA_EDEVICE;
    capacity_bytes = u64(free_b) / 2;
  }
  sa_server* srv = new (std::nothrow) sa_server();
  if (!srv) return SA_ENOMEM;
  srv->device = device;
  srv->max_text = max_text;
  // Two lanes when the size range is wide: texts up to 1 MiB share a lane with
  // a quarter of the memory; longer texts use the rest.
  const u64 small = u64(1) << 20;
  struct Spec {
    u64 cap, maxn;
  };
  std::vector<Spec> specs;
  if (max_text > 16 * small && capacity_bytes / 4 / 50 >= small) {
    specs.push_back({capacity_bytes / 4, small});
    specs.push_back({capacity_bytes - capacity_bytes / 4, max_text});
  } else {
    specs.push_back({capacity_bytes, max_text});
  }
  for (const Spec& sp : specs) {
    std::unique_ptr<Lane> L;
    sa_status st = lane_create(L, device, sp.cap, sp.maxn);
    if (st != SA_OK) {
      lane_destroy(L.get());
      sa_server_destroy(srv);
      return st;
    }
    srv->lanes.push_back(std::move(L));
    srv->lane_max.push_back(sp.maxn);
  }
  *out = srv;
  return SA_OK;
}

sa_status sa_server_destroy(sa_server* srv) {
  if (!srv) return SA_OK;
  for (auto& L : srv->lanes) lane_destroy(L.get());
  srv->lanes.clear();
  delete srv;
  return SA_OK;
}

sa_status sa_server_submit(sa_server* srv, const uint8_t* h_text, uint64_t n, uint64_t* ticket) {
  if (!srv || !ticket || (!h_text && n)) return SA_EINVAL;
  if (n > srv->max_text) return SA_ETOOBIG;
  int lane = -1;
  for (size_t k = 0; k < srv->lanes.size(); ++k)
    if (n <= srv->lane_max[k] && n <= srv->lanes[k]->arena_cap) {
      lane = int(k);
      break;
    }
  if (lane < 0) return SA_ETOOBIG;
  u64 t;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    t = srv->next_ticket++;
    srv->owner[t] = lane;
  }
  sa_status st = lane_submit(srv->lanes[lane].get(), t, h_text, n);
  if (st != SA_OK) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->owner.erase(t);
    return st;
  }
  *ticket = t;
  return SA_OK;
}

sa_status sa_server_poll(sa_server* srv, uint64_t ticket, uint32_t* h_sa_out, int* done,
                         double* latency_ms) {
  if (!srv || !done) return SA_EINVAL;
  *done = 0;
  int lane;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->owner.find(ticket);
    if (it == srv->owner.end()) return SA_EINVAL;
    lane = it->second;
  }
  bool released = false;
  sa_status st = lane_poll(srv->lanes[lane].get(), ticket, h_sa_out, done, latency_ms, &released);
  if (released) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->owner.erase(ticket);
  }
  return st;
}

sa_status sa_server_stats(sa_server* srv, sa_server_stats_t* out) {
  if (!srv || !out) return SA_EINVAL;
  std::memset(out, 0, sizeof(*out));
  for (auto& L : srv->lanes) {
    std::lock_guard<std::mutex> lk(L->mu);
    out->completed += L->completed;
    out->failed += L->failed;
    out->suffixes += L->suffixes;
    out->rounds += L->rounds;
    out->busy_ms += L->busy_s * 1e3;
    out->queued += L->queue.size();
    out->running += L->eng.live.size();
    out->slots += L->eng.slots;
    out->arena_positions += L->arena_cap;
  }
  return SA_OK;
}

}  // extern "C"
