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
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "driver.h"

using namespace drv;

namespace {

// Device tables and host mirrors of the text slots.
struct Engine {
  sa_ctx* c = nullptr;
  u32 slots = 0;
  int idbits = 0;   // slot bits at the top of every key
  int B = 0;        // bits of a rank
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
  u64 active = 0;         // survivors carried into the next round
  std::vector<u32> live;  // slots with elements in the active set or joining now

  ~Engine() { release(); }
  void release() {
    (void)hipFree(dev);
    dev = nullptr;
    if (h_wc) (void)hipHostFree(h_wc);
    if (h_surv) (void)hipHostFree(h_surv);
    h_wc = h_surv = nullptr;
  }

  sa_status init(sa_ctx* ctx, u32 nslots, int id_bits, int rank_bits) {
    c = ctx;
    slots = nslots;
    idbits = id_bits;
    B = rank_bits;
    const size_t S = nslots;
    size_t bytes = 0;
    auto take = [&](size_t b) {
      const size_t at = bytes;
      bytes += (b + 255) / 256 * 256;
      return at;
    };
    const size_t o_base = take(S * 8), o_len = take(S * 8), o_code = take(S * 256 * 2),
                 o_pres = take(S * 32), o_wc = take(S * 4), o_h = take(S * 8), o_r0 = take(S),
                 o_surv = take(S * 4), o_nt = take(S * 4), o_no = take((S + 1) * 8),
                 o_nc = take((S + 1) * 8);
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
    d_new_t = reinterpret_cast<u32*>(p + o_nt);
    d_new_out = reinterpret_cast<u64*>(p + o_no);
    d_new_chunk0 = reinterpret_cast<u64*>(p + o_nc);
    if (hipHostMalloc(reinterpret_cast<void**>(&h_wc), S * 4) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h_surv), S * 4) != hipSuccess)
      return SA_ENOMEM;
    base.assign(S, 0);
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
    const Bufs full = full_bufs(c);
    const int idshift = 64 - idbits;
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
    // Upload the tables that changed (small: a few values per slot).
    if (m) {
      if (hipMemcpyAsync(d_new_t, nt.data(), m * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(d_new_out, nout.data(), (m + 1) * 8, hipMemcpyHostToDevice, s) !=
              hipSuccess ||
          hipMemcpyAsync(d_new_chunk0, nchunk.data(), (m + 1) * 8, hipMemcpyHostToDevice, s) !=
              hipSuccess)
        return SA_EDEVICE;
    }
    if (hipMemcpyAsync(tab.base, base.data(), slots * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(tab.len, len.data(), slots * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(tab.h, h.data(), slots * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(tab.round0, round0.data(), slots, hipMemcpyHostToDevice, s) != hipSuccess)
      return SA_EDEVICE;
    // The host vectors must stay alive until the copies ran: the round ends
    // with a stream synchronisation below, and the vectors are members or
    // locals that outlive it.
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
        launch_multi_codes(tab, nl, idbits, c->round0_trim, s);
      }
      Tracer tr(c, s, SA_KERNEL_PACK_TEXT, double(A0) * 13.0);
      launch_multi_pack0(text_arena, tab, nl, idshift, c->keysA, c->valsA, s);
    }
    if (active) {
      Tracer tr(c, s, SA_KERNEL_PACK_PAIRS, double(active) * 24.0);
      launch_multi_pack_pairs(c->act_ti, c->act_rank, active, tab, B, idshift, c->isa,
                              c->keysA + A0, c->valsA + A0, s);
    }
    const u64 total = A0 + active;
    if (total) {
      run_sort(c, full, total, kMaxPasses, 1, slot_info, s);
      RerankArgs a{};
      a.count = total;
      a.n = 0;
      a.gshift = B;  // group = (slot, rank) for texts past round 0
      a.rshift = B;
      a.rmask = (u64(1) << B) - 1;
      a.idshift = idshift;
      a.mode = kRerankScatterIsa;
      a.tbase = tab.base;
      a.tlen = tab.len;
      a.tround0 = tab.round0;
      run_rerank(c, full, a, sa_arena, s);
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
};

}  // namespace

// ---------------------------------------------------------------------------
// Batched build.

struct sa_batch_state {
  Engine eng;
};

namespace {

sa_status build_batch(sa_ctx* c, const u8* text, const u64* h_off, u32 T, u32* d_sa,
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
  if (N == 0) return SA_OK;
  if (!text || !d_sa) return SA_EINVAL;
  if (T == 1) return build_rounds(c, text, N, 0, d_sa, nullptr, s);
  const int idbits = bits_of(u64(T) - 1);
  const int B = bits_of(max_n);
  if (idbits + 2 * B > 64) return SA_ETOOBIG;
  if (hipSetDevice(c->device) != hipSuccess) return SA_EDEVICE;
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
    info.passes_run[r] = passes_run(c, r, kMaxPasses);
    info.key_bits[r] = 64;
    info.rounds = u32(r + 1);
    in_round = eng.active;
    if (eng.active == 0) break;
  }
  u32 maxc = 0;
  for (u32 t = 0; t < T; ++t) maxc = std::max(maxc, eng.chars[t]);
  info.chars0 = maxc;
  info.prefix_len = u64(maxc) << (info.rounds - 1);
  return SA_OK;
}

}  // namespace

extern "C" sa_status sa_build_batch(sa_ctx* ctx, const uint8_t* d_texts,
                                    const uint64_t* h_offsets, uint32_t num_texts,
                                    uint32_t* d_sas, void* stream) {
  if (!ctx) return SA_EINVAL;
  sa_status st = build_batch(ctx, d_texts, h_offsets, num_texts, d_sas,
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
  std::vector<u8> text;  // host copy until the text is on the device
  u64 n = 0;
  double t_arrive = 0, t_admit = 0, t_done = 0;
  int state = 0;  // 0 queued, 1 running, 2 done, 3 failed, 4 being copied out
  u32 slot = 0;
  u64 base = 0;
  sa_status err = SA_OK;
};

}  // namespace

struct sa_server {
  sa_ctx* ctx = nullptr;
  Engine eng;
  int device = 0;
  u64 arena_cap = 0;  // positions
  u64 max_text = 0;
  u8* d_text = nullptr;
  u32* d_sa = nullptr;
  hipStream_t stream = nullptr;
  std::map<u64, u64> free_ranges;  // start -> length
  std::deque<u64> queue;
  std::unordered_map<u64, std::unique_ptr<Request>> reqs;
  std::vector<u32> free_slots;
  std::vector<u64> slot_ticket;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  u64 next_ticket = 1;
  // statistics
  u64 completed = 0, failed = 0, suffixes = 0, rounds = 0;
  double busy_s = 0;

  bool alloc(u64 n, u64* out) {
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second >= n) {
        *out = it->first;
        const u64 rest = it->second - n, start = it->first + n;
        free_ranges.erase(it);
        if (rest) free_ranges[start] = rest;
        return true;
      }
    }
    return false;
  }

  void release(u64 start, u64 n) {
    if (n == 0) return;
    auto it = free_ranges.emplace(start, n).first;
    auto nx = std::next(it);
    if (nx != free_ranges.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_ranges.erase(nx);
    }
    if (it != free_ranges.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_ranges.erase(it);
      }
    }
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
      for (Request* r : copies)
        if (hipMemcpyAsync(d_text + r->base, r->text.data(), r->n, hipMemcpyHostToDevice,
                           stream) != hipSuccess)
          st = SA_EDEVICE;
      if (st == SA_OK) st = eng.round_step(d_text, d_sa, joining, finished, 0, stream);
      if (st == SA_OK) {
        // The texts are on the device once the round has synchronised.
        for (Request* r : copies) std::vector<u8>().swap(r->text);
      }
      const double t1 = now_s();
      std::lock_guard<std::mutex> lk(mu);
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

extern "C" {

sa_status sa_server_create(sa_server** out, int device, uint64_t capacity_bytes,
                           uint64_t max_text) {
  if (!out) return SA_EINVAL;
  *out = nullptr;
  if (max_text == 0) max_text = u64(1) << 26;
  if (max_text >= (u64(1) << 32)) return SA_ETOOBIG;
  const int B = bits_of(max_text);
  int idbits = 64 - 2 * B;
  if (idbits < 1) return SA_ETOOBIG;
  if (idbits > 10) idbits = 10;  // at most 1024 requests in flight
  sa_server* srv = new (std::nothrow) sa_server();
  if (!srv) return SA_ENOMEM;
  srv->device = device;
  srv->max_text = max_text;
  auto fail = [srv](sa_status e) {
    sa_server_destroy(srv);  // frees whatever was set up; no worker yet
    return e;
  };
  sa_status st = sa_ctx_create(&srv->ctx, device, nullptr);
  if (st != SA_OK) return fail(st);
  if (capacity_bytes == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(SA_EDEVICE);
    capacity_bytes = u64(free_b) / 2;
  }
  // Per arena position: text 1 + SA 4 + ISA 4 + keys 16 + values 8 + survivors
  // 16 + look-back status ~1.
  const u64 per = 50;
  srv->arena_cap = capacity_bytes / per;
  if (srv->arena_cap < max_text) return fail(SA_ENOMEM);
  sa_ctx* c = srv->ctx;
  st = ensure_workspace(c, srv->arena_cap);
  if (st != SA_OK) return fail(st);
  if (!dev_alloc(&c->act_ti, c->cap)) return fail(SA_ENOMEM);
  c->act_ti_cap = c->cap;
  if (!dev_alloc(&srv->d_text, srv->arena_cap) || !dev_alloc(&srv->d_sa, srv->arena_cap))
    return fail(SA_ENOMEM);
  const u32 slots = 1u << idbits;
  st = srv->eng.init(c, slots, idbits, B);
  if (st != SA_OK) return fail(st);
  if (hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess)
    return fail(SA_EDEVICE);
  srv->free_ranges[0] = srv->arena_cap;
  srv->slot_ticket.assign(slots, 0);
  for (u32 k = slots; k-- > 0;) srv->free_slots.push_back(k);
  try {
    srv->worker = std::thread([srv] { srv->run(); });
  } catch (...) {
    return fail(SA_ENOMEM);
  }
  *out = srv;
  return SA_OK;
}

sa_status sa_server_destroy(sa_server* srv) {
  if (!srv) return SA_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  (void)hipSetDevice(srv->device);
  if (srv->stream) (void)hipStreamDestroy(srv->stream);
  (void)hipFree(srv->d_text);
  (void)hipFree(srv->d_sa);
  srv->eng.release();
  if (srv->ctx) sa_ctx_destroy(srv->ctx);
  delete srv;
  return SA_OK;
}

sa_status sa_server_submit(sa_server* srv, const uint8_t* h_text, uint64_t n, uint64_t* ticket) {
  if (!srv || !ticket || (!h_text && n)) return SA_EINVAL;
  if (n > srv->max_text || n > srv->arena_cap) return SA_ETOOBIG;
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return SA_ENOMEM;
  r->n = n;
  r->t_arrive = now_s();
  try {
    r->text.assign(h_text, h_text + n);
  } catch (...) {
    return SA_ENOMEM;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  const u64 t = srv->next_ticket++;
  if (n == 0) {
    r->state = 2;
    r->t_admit = r->t_done = r->t_arrive;
    srv->completed += 1;
  } else {
    srv->queue.push_back(t);
  }
  srv->reqs[t] = std::move(r);
  *ticket = t;
  srv->cv.notify_all();
  return SA_OK;
}

sa_status sa_server_poll(sa_server* srv, uint64_t ticket, uint32_t* h_sa_out, int* done,
                         double* latency_ms) {
  if (!srv || !done) return SA_EINVAL;
  *done = 0;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return SA_EINVAL;
    r = it->second.get();
    if (r->state == 3) {
      const sa_status e = r->err;
      srv->reqs.erase(it);
      return e;
    }
    if (r->state != 2) return SA_OK;
    if (r->n && !h_sa_out) return SA_EINVAL;
    r->state = 4;
  }
  sa_status st = SA_OK;
  if (r->n) {
    if (hipSetDevice(srv->device) != hipSuccess ||
        hipMemcpy(h_sa_out, srv->d_sa + r->base, r->n * sizeof(u32), hipMemcpyDeviceToHost) !=
            hipSuccess)
      st = SA_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (latency_ms) *latency_ms = (r->t_done - r->t_arrive) * 1e3;
  srv->release(r->base, r->n);
  srv->reqs.erase(ticket);
  srv->cv.notify_all();
  if (st == SA_OK) *done = 1;
  return st;
}

sa_status sa_server_stats(sa_server* srv, sa_server_stats_t* out) {
  if (!srv || !out) return SA_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  std::memset(out, 0, sizeof(*out));
  out->completed = srv->completed;
  out->failed = srv->failed;
  out->suffixes = srv->suffixes;
  out->rounds = srv->rounds;
  out->busy_ms = srv->busy_s * 1e3;
  out->queued = srv->queue.size();
  out->running = srv->eng.live.size();
  out->slots = srv->eng.slots;
  out->arena_positions = srv->arena_cap;
  return SA_OK;
}

}  // extern "C"
