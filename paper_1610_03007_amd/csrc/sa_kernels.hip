// gfx950 kernels for suffix-array construction by prefix doubling with
// discarding (Bingmann, Gog, Kurpicz, Section 2.1, Alg. 1, 4, 5 and 6).
//
// One doubling round is: build keys (round 0 from the text, later rounds from
// the current rank and the rank h positions on), stable LSD radix sort of
// (key, text position) pairs, then one fused pass that re-ranks, scatters the
// inverse suffix array, writes final SA entries of suffixes whose rank became
// unique and compacts the rest into the next round's active list.
//
// All arithmetic is integer. Every kernel is wave64; cross-workgroup scans use
// decoupled look-back over tiles taken from an atomic ticket, so a tile only
// ever waits for tiles that are already running; every wait is bounded.

#include "kernels.h"

namespace sa {

namespace {

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ inline u32 wave_inclusive_sum(u32 v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    u32 t = __shfl_up(v, off, kWave);
    if (lane >= off) v += t;
  }
  return v;
}

__device__ inline u64 wave_inclusive_sum64(u64 v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    u64 t = __shfl_up(v, off, kWave);
    if (lane >= off) v += t;
  }
  return v;
}

__device__ inline u64 wave_inclusive_max64(u64 v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    u64 t = __shfl_up(v, off, kWave);
    if (lane >= off) v = t > v ? t : v;
  }
  return v;
}

// Look back over earlier tiles of a single-pass scan and return the exclusive
// prefix for `tile` (tile > 0). `op_max` selects max instead of sum. Publishes
// the inclusive prefix. Bounded: on time-out raises kErrLookbackTimeout and
// sets *timed_out (an LDS flag) so that the workgroup writes nothing.
__device__ u64 lookback(u64* status, u64 stride, u64 tile, u64 agg, u32 gen, bool op_max,
                        u64* counters, u32* timed_out) {
  u64 excl = 0;
  u64 t = tile - 1;
  u32 spins = 0;
  for (;;) {
    u64 s = load_status(status + t * stride);
    u32 f = status_flag(s);
    if (status_gen(s) != (gen & kGenMask) || f == 0) {
      if (++spins > kSpinLimit) {
        atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
                 (unsigned long long)kErrLookbackTimeout);
        *timed_out = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    u64 v = status_value(s);
    excl = op_max ? (v > excl ? v : excl) : excl + v;
    if (f == kFlagPrefix || t == 0) break;
    --t;
  }
  u64 inc = op_max ? (agg > excl ? agg : excl) : excl + agg;
  store_status(status + tile * stride, status_pack(gen, kFlagPrefix, inc));
  return excl;
}

}  // namespace

// ---------------------------------------------------------------------------
// Small utility kernels.

__global__ void fill_u64_kernel(u64* p, u64 count, u64 value) {
  u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

void launch_fill_u64(u64* p, u64 count, u64 value, hipStream_t s) {
  if (count == 0) return;
  u64 blocks = ceil_div(count, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(u32(blocks)), dim3(256), 0, s, p, count, value);
}

__global__ void set_zero_u32_kernel(u32* p) { p[0] = 0; }

void launch_set_zero_u32(u32* p, hipStream_t s) {
  hipLaunchKernelGGL(set_zero_u32_kernel, dim3(1), dim3(1), 0, s, p);
}

// ---------------------------------------------------------------------------
// Alphabet reduction. Characters are re-coded densely as 1..sigma in byte order
// so that 0 stays free for the end-of-text sentinel (which the paper requires
// to compare below every character) and a round-0 key holds as many
// characters as fit in 64 bits.

__global__ __launch_bounds__(256) void byte_presence_kernel(const u8* __restrict__ text, u64 n,
                                                            int vec_ok, u32* __restrict__ present) {
  __shared__ u32 seen[256];
  seen[threadIdx.x] = 0;
  __syncthreads();
  const u64 nvec = vec_ok ? n / 16 : 0;
  const uint4* v = reinterpret_cast<const uint4*>(text);
  u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < nvec; i += stride) {
    uint4 w = v[i];
    u32 words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int b = 0; b < 4; ++b) seen[(words[q] >> (8 * b)) & 0xFF] = 1;
    }
  }
  for (u64 i = nvec * 16 + u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    seen[text[i]] = 1;
  __syncthreads();
  if (seen[threadIdx.x]) atomicOr(&present[threadIdx.x], 1u);
}

void launch_byte_presence(const u8* text, u64 n, u32* present, hipStream_t s) {
  u64 blocks = ceil_div(n, 256 * 16 * 8);
  if (blocks < 1) blocks = 1;
  if (blocks > 2048) blocks = 2048;
  int vec_ok = (reinterpret_cast<uintptr_t>(text) & 15) == 0;
  hipLaunchKernelGGL(byte_presence_kernel, dim3(u32(blocks)), dim3(256), 0, s, text, n, vec_ok,
                     present);
}

__global__ __launch_bounds__(256) void alphabet_codes_kernel(const u32* __restrict__ present,
                                                             u16* __restrict__ code,
                                                             u64* __restrict__ counters) {
  __shared__ u32 wsum[4];
  const int t = threadIdx.x;
  u32 p = present[t] ? 1u : 0u;
  u32 inc = wave_inclusive_sum(p);
  if (lane_id() == kWave - 1) wsum[t / kWave] = inc;
  __syncthreads();
  u32 off = 0, total = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < t / kWave) off += wsum[w];
    total += wsum[w];
  }
  u32 excl = off + inc - p;
  code[t] = p ? u16(excl + 1) : u16(0);
  if (t == 0) {
    u32 sigma = total;
    u32 w = 32 - __clz(sigma);  // bits of sigma: codes 1..sigma, 0 = sentinel
    if (w == 0) w = 1;
    counters[kCtrSigma] = sigma;
    counters[kCtrCodeBits] = w;
    counters[kCtrChars] = 64 / w;
  }
}

void launch_alphabet_codes(const u32* present, u16* code, u64* counters, hipStream_t s) {
  hipLaunchKernelGGL(alphabet_codes_kernel, dim3(1), dim3(256), 0, s, present, code, counters);
}

// ---------------------------------------------------------------------------
// Round-0 keys (the paper's initial name pairs, widened to c characters).
// A workgroup stages the codes of its window of text in LDS and each thread
// slides a c-character window over kPackItems consecutive positions.

constexpr int kPackBlock = 256;
constexpr int kPackItems = 8;
constexpr int kPackTile = kPackBlock * kPackItems;
constexpr int kPackHalo = 64;  // c <= 64

__global__ __launch_bounds__(kPackBlock) void pack_text_kernel(const u8* __restrict__ text, u64 n,
                                                               const u16* __restrict__ code,
                                                               const u64* __restrict__ counters,
                                                               u64* __restrict__ keys) {
  __shared__ u16 s_code[256];
  __shared__ u16 s_sym[kPackTile + kPackHalo];
  __shared__ u64 s_out[kPackTile];
  const int t = threadIdx.x;
  const u64 base = u64(blockIdx.x) * kPackTile;
  const u32 w = u32(counters[kCtrCodeBits]);
  const u32 c = u32(counters[kCtrChars]);
  s_code[t] = code[t];
  __syncthreads();
  for (int i = t; i < kPackTile + kPackHalo; i += kPackBlock) {
    u64 p = base + u64(i);
    s_sym[i] = (p < n) ? s_code[text[p]] : u16(0);
  }
  __syncthreads();
  const u64 keymask = (c * w >= 64) ? ~u64(0) : ((u64(1) << (c * w)) - 1);
  const int first = t * kPackItems;
  u64 key = 0;
  for (u32 j = 0; j < c; ++j) key = (key << w) | u64(s_sym[first + int(j)]);
  s_out[first] = key;
#pragma unroll
  for (int j = 1; j < kPackItems; ++j) {
    key = ((key << w) | u64(s_sym[first + j + int(c) - 1])) & keymask;
    s_out[first + j] = key;
  }
  __syncthreads();
  for (int i = t; i < kPackTile; i += kPackBlock) {
    u64 p = base + u64(i);
    if (p < n) keys[p] = s_out[i];
  }
}

void launch_pack_text(const u8* text, u64 n, const u16* code, const u64* counters, u64* keys,
                      hipStream_t s) {
  u64 blocks = ceil_div(n, kPackTile);
  hipLaunchKernelGGL(pack_text_kernel, dim3(u32(blocks)), dim3(kPackBlock), 0, s, text, n, code,
                     counters, keys);
}

// ---------------------------------------------------------------------------
// Round >= 1 keys: the name pair (own rank, rank of the suffix h positions on)
// read from the partial inverse suffix array, 0 past the end (Alg. 4 pairing).

__global__ __launch_bounds__(256) void pack_pairs_kernel(const u32* __restrict__ act_idx,
                                                         const u32* __restrict__ act_rank,
                                                         u64 count, u64 n, u64 h, int b,
                                                         const u32* __restrict__ isa,
                                                         u64* __restrict__ keys,
                                                         u32* __restrict__ vals) {
  u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= count) return;
  u32 i = act_idx[p];
  u32 r = act_rank[p];
  u64 j = u64(i) + h;
  u32 r1 = (j < n) ? isa[j] : 0u;
  keys[p] = (u64(r) << b) | u64(r1);
  vals[p] = i;
}

void launch_pack_pairs(const u32* act_idx, const u32* act_rank, u64 count, u64 n, u64 h, int b,
                       const u32* isa, u64* keys, u32* vals, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(pack_pairs_kernel, dim3(u32(ceil_div(count, 256))), dim3(256), 0, s, act_idx,
                     act_rank, count, n, h, b, isa, keys, vals);
}

// ---------------------------------------------------------------------------
// LSD radix sort, one sweep per digit (decoupled look-back across tiles).

constexpr int kHistItems = 8;

__global__ __launch_bounds__(kHistBlock) void radix_histogram_kernel(const u64* __restrict__ keys,
                                                                     u64 count, int npass,
                                                                     u64* __restrict__ hist) {
  __shared__ u32 lh[kMaxPasses * kRadix];
  for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += kHistBlock) lh[i] = 0;
  __syncthreads();
  const int lane = lane_id();
  const u64 chunk = u64(kHistBlock) * kHistItems;
  for (u64 base = u64(blockIdx.x) * chunk; base < count; base += u64(gridDim.x) * chunk) {
    u64 key[kHistItems];
    bool valid[kHistItems];
#pragma unroll
    for (int j = 0; j < kHistItems; ++j) {
      u64 e = base + u64(j) * kHistBlock + threadIdx.x;
      valid[j] = e < count;
      key[j] = valid[j] ? keys[e] : 0;
    }
#pragma unroll
    for (int j = 0; j < kHistItems; ++j) {
      const u64 vmask = __ballot(valid[j]);
      if (vmask == 0) continue;  // wave-uniform
      for (int p = 0; p < npass; ++p) {
        u32 d = u32(key[j] >> (p * kRadixBits)) & (kRadix - 1);
        // Valid lanes form a prefix of the wave, so lane 0 is valid here.
        u32 d0 = __shfl(d, 0, kWave);
        const u64 same = __ballot(valid[j] && d == d0);
        if (same == vmask) {
          if (lane == 0) atomicAdd(&lh[p * kRadix + d0], u32(__popcll(vmask)));
        } else if (valid[j]) {
          atomicAdd(&lh[p * kRadix + d], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npass * kRadix; i += kHistBlock) {
    u32 v = lh[i];
    if (v) atomicAdd(reinterpret_cast<unsigned long long*>(hist + i), (unsigned long long)v);
  }
}

void launch_radix_histogram(const u64* keys, u64 count, int npass, u64* hist, hipStream_t s) {
  if (count == 0) return;
  u64 blocks = ceil_div(count, u64(kHistBlock) * kHistItems * 4);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(radix_histogram_kernel, dim3(u32(blocks)), dim3(kHistBlock), 0, s, keys,
                     count, npass, hist);
}


// Exclusive digit offsets per pass, constant-digit passes marked skipped, and
// the ping-pong schedule of the passes that run. One workgroup, one thread per
// digit value.
__global__ __launch_bounds__(kRadix) void radix_plan_kernel(const u64* __restrict__ hist,
                                                            u64 count, int npass, int vals_present,
                                                            SortPlan* __restrict__ plan) {
  __shared__ u64 sc[kMaxPasses][kRadix];
  __shared__ u32 s_skip[kMaxPasses];
  const int d = threadIdx.x;
  if (d < kMaxPasses) s_skip[d] = 0;
  __syncthreads();
  u64 own[kMaxPasses];
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) {
    own[p] = (p < npass) ? hist[p * kRadix + d] : 0;
    sc[p][d] = own[p];
    if (p < npass && own[p] == count) s_skip[p] = 1;  // one digit holds every key
  }
  __syncthreads();
  // Hillis-Steele inclusive scans over the digits of every pass at once.
  for (int off = 1; off < kRadix; off <<= 1) {
    u64 add[kMaxPasses];
#pragma unroll
    for (int p = 0; p < kMaxPasses; ++p) add[p] = (d >= off) ? sc[p][d - off] : 0;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kMaxPasses; ++p) sc[p][d] += add[p];
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) plan->offsets[p][d] = sc[p][d] - own[p];
  if (d == 0) {
    u32 cur = 0;
    bool first = true;
    for (int p = 0; p < kMaxPasses; ++p) {
      bool run = (p < npass) && !s_skip[p];
      plan->skip[p] = run ? 0u : 1u;
      plan->src[p] = cur;
      plan->iota[p] = 0;
      if (run) {
        plan->iota[p] = (!vals_present && first) ? 1u : 0u;
        first = false;
        cur ^= 1u;
      }
    }
    if (first) {
      // Every digit is constant (all keys equal): run the top pass anyway; it
      // is a stable copy that also materialises generated values.
      int p = npass - 1;
      plan->skip[p] = 0;
      plan->src[p] = 0;
      plan->iota[p] = vals_present ? 0u : 1u;
      cur = 1;
    }
    plan->final_buf = cur;
  }
}

void launch_radix_plan(const u64* hist, u64 count, int npass, int vals_present, SortPlan* plan,
                       hipStream_t s) {
  hipLaunchKernelGGL(radix_plan_kernel, dim3(1), dim3(kRadix), 0, s, hist, count, npass,
                     vals_present, plan);
}

// One stable counting pass over digit `pass`. Per tile: load 16 items per
// thread in wave-striped order, rank every item among equal digits of its wave
// with eight ballots (the match mask) and a per-wave LDS counter, combine the
// waves, publish the tile's digit counts, look back for the counts of earlier
// tiles, reorder the tile by digit in LDS and write each digit's run out
// contiguously.
__global__ __launch_bounds__(kSortBlock) void onesweep_pass_kernel(
    u64* __restrict__ keysA, u64* __restrict__ keysB, u32* __restrict__ valsA,
    u32* __restrict__ valsB, u64 count, int pass, const SortPlan* __restrict__ plan,
    u64* __restrict__ status, u64* __restrict__ counters, u32 gen) {
  static_assert(kSortBlock == kRadix, "one thread per digit value");
  constexpr int NW = kSortBlock / kWave;
  __shared__ u64 s_keys[kSortTile];
  __shared__ u32 s_vals[kSortTile];
  __shared__ u32 s_cnt[NW][kRadix];
  __shared__ u32 s_start[kRadix];
  __shared__ u64 s_base[kRadix];
  __shared__ u32 s_wsum[NW];
  __shared__ u64 s_tile;
  __shared__ u32 s_abort;

  if (plan->skip[pass]) return;
  const u32 src = plan->src[pass];
  const bool iota = plan->iota[pass] != 0;
  const u64* kin = src ? keysB : keysA;
  u64* kout = src ? keysA : keysB;
  const u32* vin = src ? valsB : valsA;
  u32* vout = src ? valsA : valsB;
  const int shift = pass * kRadixBits;

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  if (tid == 0) {
    s_tile = atomicAdd(reinterpret_cast<unsigned long long*>(counters + kCtrSortTiles + pass),
                       1ull);
    s_abort = 0;
  }
#pragma unroll
  for (int w = 0; w < NW; ++w) s_cnt[w][tid] = 0;
  __syncthreads();
  const u64 tile = s_tile;
  const u64 tile_base = tile * kSortTile;
  const u64 wave_base = tile_base + u64(wave) * (kSortItems * kWave);

  u64 key[kSortItems];
  u32 val[kSortItems];
  u32 rank[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    u64 e = wave_base + u64(j) * kWave + lane;
    if (e < count) {
      key[j] = kin[e];
      val[j] = iota ? u32(e) : vin[e];
    } else {
      key[j] = ~u64(0);  // digit 255: lands after every valid item of the tile
      val[j] = 0;
    }
  }

  // Rank within the wave, items taken in (j, lane) order == input order. The
  // counters are read by every lane and bumped by the lowest lane of each
  // digit's match set; volatile keeps every access a real LDS access, which a
  // wave issues in program order.
  volatile u32* cnt = &s_cnt[wave][0];
  const u64 lt_mask = (u64(1) << lane) - 1;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const u32 d = u32(key[j] >> shift) & (kRadix - 1);
    u64 peers = ~u64(0);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const u64 bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const u32 below = __popcll(peers & lt_mask);
    const u32 old = cnt[d];
    if (below == 0) cnt[d] = old + u32(__popcll(peers));
    rank[j] = old + below;
  }
  __syncthreads();

  // Per digit (one per thread): exclusive prefix over waves, tile total.
  u32 tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    u32 c = s_cnt[w][tid];
    s_cnt[w][tid] = tot;
    tot += c;
  }
  u64* my_status = status + tile * kRadix + tid;
  if (tile == 0)
    store_status(my_status, status_pack(gen, kFlagPrefix, tot));
  else
    store_status(my_status, status_pack(gen, kFlagAggregate, tot));

  // Exclusive scan of the tile totals over digits: tile-local run starts.
  const u32 inc = wave_inclusive_sum(tot);
  if (lane == kWave - 1) s_wsum[wave] = inc;
  __syncthreads();
  u32 woff = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w)
    if (w < wave) woff += s_wsum[w];
  const u32 start = woff + inc - tot;
  s_start[tid] = start;

  u64 excl = 0;
  if (tile > 0) excl = lookback(status + tid, kRadix, tile, tot, gen, false, counters, &s_abort);
  s_base[tid] = plan->offsets[pass][tid] + excl - u64(start);
  __syncthreads();

#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const u32 d = u32(key[j] >> shift) & (kRadix - 1);
    const u32 q = s_start[d] + s_cnt[wave][d] + rank[j];
    s_keys[q] = key[j];
    s_vals[q] = val[j];
  }
  __syncthreads();

  if (s_abort) return;
  const u64 left = count - tile_base;
  const u32 valid = left < u64(kSortTile) ? u32(left) : u32(kSortTile);
  for (u32 q = tid; q < valid; q += kSortBlock) {
    const u64 k = s_keys[q];
    const u32 d = u32(k >> shift) & (kRadix - 1);
    const u64 o = s_base[d] + q;
    if (o < count) {
      kout[o] = k;
      vout[o] = s_vals[q];
    } else {
      atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
               (unsigned long long)kErrBounds);
    }
  }
}

void launch_onesweep_pass(u64* keysA, u64* keysB, u32* valsA, u32* valsB, u64 count, int pass,
                          const SortPlan* plan, u64* status, u64* counters, u32 gen,
                          hipStream_t s) {
  if (count == 0) return;
  const u64 tiles = ceil_div(count, kSortTile);
  hipLaunchKernelGGL(onesweep_pass_kernel, dim3(u32(tiles)), dim3(kSortBlock), 0, s, keysA, keysB,
                     valsA, valsB, count, pass, plan, status, counters, gen);
}

// ---------------------------------------------------------------------------
// Re-rank, ISA scatter, finalisation and compaction (one pass over the sorted
// active set).
//
// For element p of the sorted active set with key (r0, r1):
//   head[p]  = p is the first of its run of equal keys (the paper's name
//              comparison, Alg. 2),
//   grp[p]   = p is the first of its run of equal r0 (its group),
//   ss(p)    = last head position <= p, gs(p) = last group start <= p (both a
//              max-prefix-sum, Alg. 1 / Alg. 5),
//   newrank  = r0 + ss(p) - gs(p)  (old name plus the offset of the sub-group in
//              the group: the renaming of Alg. 6, with 1-based names).
// In round 0 every element starts in one group with r0 = 1.
// An element is unique when it is a head and the next element is a head too
// (Alg. 6 `Unique`); its rank is final, so SA[newrank - 1] = its position and it
// is discarded. All others survive, in sorted order. Every element's new rank
// goes to ISA[text position] because any suffix may be gathered later.
__global__ __launch_bounds__(kRerankBlock) void rerank_compact_kernel(
    const u64* __restrict__ keysA, const u64* __restrict__ keysB,
    const u32* __restrict__ valsA, const u32* __restrict__ valsB,
    const SortPlan* __restrict__ plan, u64 count, u64 n, int b, u32* __restrict__ isa,
    u32* __restrict__ sa_out, u32* __restrict__ act_idx, u32* __restrict__ act_rank,
    u64* __restrict__ st_head, u64* __restrict__ st_grp, u64* __restrict__ st_surv,
    u64* __restrict__ counters, u32 gen) {
  constexpr int NW = kRerankBlock / kWave;
  constexpr int T = kRerankTile;
  constexpr int I = kRerankItems;
  __shared__ u64 s_k[T + 2];
  __shared__ u32 s_v[T];
  __shared__ u64 s_wh[NW], s_wg[NW], s_ws[NW];
  __shared__ u64 s_prefix[3];
  __shared__ u64 s_tile;
  __shared__ u32 s_abort;

  const u32 fb = plan->final_buf;
  const u64* keys = fb ? keysB : keysA;
  const u32* vals = fb ? valsB : valsA;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  if (tid == 0) {
    s_tile = atomicAdd(reinterpret_cast<unsigned long long*>(counters + kCtrRerankTiles), 1ull);
    s_abort = 0;
  }
  __syncthreads();
  const u64 tile = s_tile;
  const u64 base = tile * T;

  for (int i = tid; i < T; i += kRerankBlock) {
    u64 p = base + u64(i);
    s_k[i + 1] = (p < count) ? keys[p] : 0;
    s_v[i] = (p < count) ? vals[p] : 0;
  }
  if (tid == 0) s_k[0] = (base > 0) ? keys[base - 1] : 0;
  if (tid == 1) s_k[T + 1] = (base + T < count) ? keys[base + T] : 0;
  __syncthreads();

  // Thread-local flags over I consecutive elements.
  const int first = tid * I;
  u64 th_head = 0, th_grp = 0, th_surv = 0;  // max head pos, max group pos, survivors
  u32 flags = 0;                             // bit j: head, bit 8+j: grp, bit 16+j: unique
#pragma unroll
  for (int j = 0; j < I; ++j) {
    const u64 p = base + u64(first + j);
    if (p >= count) break;
    const u64 k = s_k[first + j + 1];
    const u64 kp = s_k[first + j];
    const u64 kn = s_k[first + j + 2];
    const bool head = (p == 0) || (k != kp);
    const bool grp = (p == 0) || (b > 0 && (k >> b) != (kp >> b));
    const bool next_head = (p + 1 == count) || (kn != k);
    const bool uniq = head && next_head;
    if (head) {
      th_head = p;
      flags |= 1u << j;
    }
    if (grp) {
      th_grp = p;
      flags |= 1u << (8 + j);
    }
    if (uniq) flags |= 1u << (16 + j);
    else th_surv += 1;
  }

  // Block-wide scans: inclusive max for heads and groups, inclusive sum for survivors.
  const u64 ih = wave_inclusive_max64(th_head);
  const u64 ig = wave_inclusive_max64(th_grp);
  const u64 is = wave_inclusive_sum64(th_surv);
  if (lane == kWave - 1) {
    s_wh[wave] = ih;
    s_wg[wave] = ig;
    s_ws[wave] = is;
  }
  __syncthreads();
  u64 bh = 0, bg = 0, bs = 0;        // exclusive over earlier waves
  u64 tot_h = 0, tot_g = 0, tot_s = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wave) {
      bh = s_wh[w] > bh ? s_wh[w] : bh;
      bg = s_wg[w] > bg ? s_wg[w] : bg;
      bs += s_ws[w];
    }
    tot_h = s_wh[w] > tot_h ? s_wh[w] : tot_h;
    tot_g = s_wg[w] > tot_g ? s_wg[w] : tot_g;
    tot_s += s_ws[w];
  }
  // Exclusive within the block for this thread.
  u64 eh = __shfl_up(ih, 1, kWave);
  u64 eg = __shfl_up(ig, 1, kWave);
  u64 es = is - th_surv;
  if (lane == 0) {
    eh = 0;
    eg = 0;
  }
  eh = eh > bh ? eh : bh;
  eg = eg > bg ? eg : bg;
  es += bs;

  // Tile prefixes from earlier tiles (threads 0..2 of wave 0 look back).
  if (tid < 3) {
    u64* st = tid == 0 ? st_head : (tid == 1 ? st_grp : st_surv);
    const u64 agg = tid == 0 ? tot_h : (tid == 1 ? tot_g : tot_s);
    u64 pre = 0;
    if (tile == 0)
      store_status(st, status_pack(gen, kFlagPrefix, agg));
    else {
      store_status(st + tile, status_pack(gen, kFlagAggregate, agg));
      pre = lookback(st, 1, tile, agg, gen, tid != 2, counters, &s_abort);
    }
    s_prefix[tid] = pre;
    if (tid == 2 && base + T >= count) counters[kCtrActive] = pre + agg;  // last tile
  }
  __syncthreads();
  if (s_abort) return;
  u64 ss = s_prefix[0] > eh ? s_prefix[0] : eh;
  u64 gs = s_prefix[1] > eg ? s_prefix[1] : eg;
  u64 out = s_prefix[2] + es;

#pragma unroll
  for (int j = 0; j < I; ++j) {
    const u64 p = base + u64(first + j);
    if (p >= count) break;
    if (flags & (1u << j)) ss = p;
    if (flags & (1u << (8 + j))) gs = p;
    const u64 k = s_k[first + j + 1];
    const u32 v = s_v[first + j];
    const u64 r0 = b > 0 ? (k >> b) : 1;
    const u64 nr = r0 + ss - gs;
    if (v >= n || nr == 0 || nr > n || out >= count) {
      atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
               (unsigned long long)kErrBounds);
      break;
    }
    isa[v] = u32(nr);
    if (flags & (1u << (16 + j))) {
      sa_out[nr - 1] = v;
    } else {
      act_idx[out] = v;
      act_rank[out] = u32(nr);
      ++out;
    }
  }
}

void launch_rerank_compact(const u64* keysA, const u64* keysB, const u32* valsA,
                           const u32* valsB, const SortPlan* plan, u64 count, u64 n, int b,
                           u32* isa, u32* sa_out, u32* act_idx, u32* act_rank, u64* st_head,
                           u64* st_grp, u64* st_surv, u64* counters, u32 gen, hipStream_t s) {
  if (count == 0) return;
  const u64 tiles = ceil_div(count, kRerankTile);
  hipLaunchKernelGGL(rerank_compact_kernel, dim3(u32(tiles)), dim3(kRerankBlock), 0, s, keysA,
                     keysB, valsA, valsB, plan, count, n, b, isa, sa_out, act_idx, act_rank, st_head,
                     st_grp, st_surv, counters, gen);
}

}  // namespace sa
