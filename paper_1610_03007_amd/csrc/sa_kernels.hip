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

#include <atomic>

#include "kernels.h"

namespace sa {

namespace {

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

// The RB-bit digit at bit `shift` (a multiple of RB, the same in every lane)
// of a key. Byte digits never straddle the two 32-bit words: the word that
// holds the digit, then a bit-field extract; other widths shift the key.
template <int RB>
__device__ inline u32 digit_at(u64 k, int shift) {
  if constexpr (RB == 8) {
    const u32 word = shift >= 32 ? u32(k >> 32) : u32(k);
    return __builtin_amdgcn_ubfe(word, u32(shift & 31), 8u);
  } else {
    return u32(k >> shift) & ((1u << RB) - 1u);
  }
}


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

__global__ void fill_u32_kernel(u32* p, u64 count, u32 value) {
  u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

void launch_fill_u32(u32* p, u64 count, u32 value, hipStream_t s) {
  if (count == 0) return;
  u64 blocks = ceil_div(count, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(u32(blocks)), dim3(256), 0, s, p, count, value);
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

// Bytes present: every lane stores 1 into an LDS table entry per byte value it
// reads (stores of one instruction to the same entry do not serialise), and
// the table is ORed into the global one.
__global__ __launch_bounds__(256) void byte_presence_kernel(const u8* __restrict__ text, u64 n,
                                                            int vec_ok, u32* __restrict__ present) {
  __shared__ u32 seen[256];
  seen[threadIdx.x] = 0;
  __syncthreads();
  const u64 nvec = vec_ok ? n / 16 : 0;
  const uint4* v = reinterpret_cast<const uint4*>(text);
  u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < nvec; i += stride) {
    const uint4 w = v[i];
    const u32 words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int b = 0; b < 4; ++b) seen[(words[q] >> (8 * b)) & 0xFFu] = 1;
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
                                                             u64* __restrict__ counters,
                                                             int trim, int idbits, int rb) {
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
    // As many characters as fit in 64 bits; with `trim`, drop the characters
    // that would only half-fill a last rb-bit radix digit, saving one sort pass
    // over every suffix for a slightly shorter first prefix.
    // `idbits` high key bits are taken by a text id (batches).
    const u32 avail = 64u - u32(idbits);
    u32 c = avail / w;
    if (c < 1) c = 1;
    const u32 used = u32(idbits) + c * w;
    const u32 urb = u32(rb);
    if (trim && used % urb != 0 && used > urb) {
      const u32 full = (used / urb) * urb;
      if (full > u32(idbits)) {
        const u32 ct = (full - u32(idbits)) / w;
        if (ct >= 1) c = ct;
      }
    }
    counters[kCtrSigma] = sigma;
    counters[kCtrCodeBits] = w;
    counters[kCtrChars] = c;
  }
}

void launch_alphabet_codes(const u32* present, u16* code, u64* counters, int trim, int idbits,
                           int rb, hipStream_t s) {
  hipLaunchKernelGGL(alphabet_codes_kernel, dim3(1), dim3(256), 0, s, present, code, counters,
                     trim, idbits, rb);
}

// ---------------------------------------------------------------------------
// Round-0 keys (the paper's initial name pairs, widened to c characters).
// A workgroup stages the codes of its window of text in LDS and each thread
// slides a c-character window over kPackItems consecutive positions.

constexpr int kPackBlock = 256;
constexpr int kPackItems = 8;  // multi-text packing: one 2048-position chunk per workgroup
constexpr int kPackTile = kPackBlock * kPackItems;
constexpr int kPackHalo = 64;  // c <= 64
constexpr int kPackTextItems = 16;  // single text
constexpr int kPackTextTile = kPackBlock * kPackTextItems;

// LDS index of item j of thread t in a [threads][items] key array padded to
// items + 1 per thread, so that both the per-thread writes (stride items + 1
// words of 8 bytes) and the coalesced reads spread over the banks.
template <int ITEMS>
__device__ inline int pad_out(int t, int j) {
  return t * (ITEMS + 1) + j;
}

// Round-0 keys: thread t rolls the keys of kPackTextItems consecutive positions
// (c codes for the first, one more for each next key) from the tile's codes
// staged in LDS; the keys leave through LDS in coalesced order. The text is
// read as 4-byte words when it is 4-byte aligned.
__global__ __launch_bounds__(kPackBlock) void pack_text_kernel(const u8* __restrict__ text, u64 n,
                                                               int words,
                                                               const u16* __restrict__ code,
                                                               const u64* __restrict__ counters,
                                                               u64* __restrict__ keys) {
  constexpr int IT = kPackTextItems;
  constexpr int TILE = kPackTextTile;
  __shared__ u16 s_code[256];
  __shared__ u16 s_sym[TILE + kPackHalo];
  __shared__ u64 s_out[kPackBlock * (IT + 1)];
  const int t = threadIdx.x;
  const u64 base = u64(blockIdx.x) * TILE;
  const u32 w = u32(counters[kCtrCodeBits]);
  const u32 c = u32(counters[kCtrChars]);
  s_code[t] = code[t];
  __syncthreads();
  if (words && base + TILE + kPackHalo <= n) {
    const u32* tw = reinterpret_cast<const u32*>(text + base);
    for (int q = t; q < (TILE + kPackHalo) / 4; q += kPackBlock) {
      const u32 v = tw[q];
      s_sym[4 * q] = s_code[v & 0xFFu];
      s_sym[4 * q + 1] = s_code[(v >> 8) & 0xFFu];
      s_sym[4 * q + 2] = s_code[(v >> 16) & 0xFFu];
      s_sym[4 * q + 3] = s_code[v >> 24];
    }
  } else {
    for (int i = t; i < TILE + kPackHalo; i += kPackBlock) {
      const u64 p = base + u64(i);
      s_sym[i] = (p < n) ? s_code[text[p]] : u16(0);
    }
  }
  __syncthreads();
  const u64 keymask = (c * w >= 64) ? ~u64(0) : ((u64(1) << (c * w)) - 1);
  const int first = t * IT;
  u64 key = 0;
  for (u32 j = 0; j < c; ++j) key = (key << w) | u64(s_sym[first + int(j)]);
  s_out[pad_out<IT>(t, 0)] = key;
#pragma unroll
  for (int j = 1; j < IT; ++j) {
    key = ((key << w) | u64(s_sym[first + j + int(c) - 1])) & keymask;
    s_out[pad_out<IT>(t, j)] = key;
  }
  __syncthreads();
  // Position i of the tile is item i % IT of thread i / IT.
  if (base + TILE <= n) {
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const int i = j * kPackBlock + t;
      // Written once and read by the next kernel: non-temporal.
      __builtin_nontemporal_store(s_out[pad_out<IT>(i / IT, i % IT)], keys + base + u64(i));
    }
  } else {
    for (int i = t; i < TILE; i += kPackBlock) {
      const u64 p = base + u64(i);
      if (p < n) keys[p] = s_out[pad_out<IT>(i / IT, i % IT)];
    }
  }
}

void launch_pack_text(const u8* text, u64 n, const u16* code, const u64* counters, u64* keys,
                      hipStream_t s) {
  u64 blocks = ceil_div(n, kPackTextTile);
  const int words = (reinterpret_cast<uintptr_t>(text) & 3) == 0 ? 1 : 0;
  hipLaunchKernelGGL(pack_text_kernel, dim3(u32(blocks)), dim3(kPackBlock), 0, s, text, n, words,
                     code, counters, keys);
}

// ---------------------------------------------------------------------------
// Round >= 1 keys: the name pair (own rank, rank of the suffix h positions on)
// read from the partial inverse suffix array, 0 past the end (Alg. 4 pairing).

__global__ __launch_bounds__(256) void pack_pairs_kernel(const u32* __restrict__ act_idx,
                                                         const u32* __restrict__ act_rank,
                                                         const SortCtl* __restrict__ ctl,
                                                         const RoundCtl* __restrict__ rc, u64 n,
                                                         int b, const u32* __restrict__ isa,
                                                         u64* __restrict__ keys,
                                                         u32* __restrict__ vals) {
  const u64 count = ctl->count;
  const u64 h = rc->h;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  if (ctl->dense) {
    // Both names are read in position order: two streams, no gather.
    for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
      const u64 j = i + h;
      const u32 r1 = (j < n) ? isa[j] : 0u;
      keys[i] = (u64(isa[i]) << b) | u64(r1);
    }
    return;
  }
  for (u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x; p < count; p += stride) {
    const u32 i = act_idx[p];
    const u32 r = act_rank[p];
    const u64 j = u64(i) + h;
    const u32 r1 = (j < n) ? isa[j] : 0u;
    keys[p] = (u64(r) << b) | u64(r1);
    vals[p] = i;
  }
}

void launch_pack_pairs(const u32* act_idx, const u32* act_rank, const SortCtl* ctl,
                       const RoundCtl* rc, u64 n, int b, const u32* isa, u64* keys, u32* vals,
                       u32 grid, hipStream_t s) {
  hipLaunchKernelGGL(pack_pairs_kernel, dim3(grid), dim3(256), 0, s, act_idx, act_rank, ctl, rc, n,
                     b, isa, keys, vals);
}

// ---------------------------------------------------------------------------
// Prefix quadrupling (Section 2.1): a round sorts the rank quadruples
// (r0, r1, r2, r3) = (ISA[i], ISA[i+h], ISA[i+2h], ISA[i+3h]) (0 past the end)
// and resolves prefix length 4h. The 4b-bit key is sorted as two 2b-bit words,
// least significant first (LSD order across the words):
//   1. lo = r2 << b | r3 for every sorted suffix, values = position;
//   2. sort; name the runs of equal lo (1 + the run's first sorted position),
//      written with the position as pk[q] = lname << 32 | i in sorted order;
//   3. hi = r0 << b | r1 in that order;
//   4. stable sort of hi with generated values q (the lo-sorted index);
//   5. permute: position and lname of each hi-sorted element, read through q;
//   6. re-rank with (hi, lname) as the key, hi's upper half as the group.
// lname increases with lo, so (hi, lname) orders like (r0, r1, r2, r3).

__device__ inline u32 isa_or_zero(const u32* __restrict__ isa, u64 j, u64 n) {
  return j < n ? isa[j] : 0u;
}

__global__ __launch_bounds__(256) void pack_quad_lo_kernel(const u32* __restrict__ act_idx,
                                                           const SortCtl* __restrict__ ctl,
                                                           const RoundCtl* __restrict__ rc, u64 n,
                                                           int b, const u32* __restrict__ isa,
                                                           u64* __restrict__ keys,
                                                           u32* __restrict__ vals) {
  const u64 count = ctl->count;
  const u64 h = rc->h;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  const bool dense = ctl->dense != 0;
  for (u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x; p < count; p += stride) {
    // A dense round takes every position in order (the sort generates the
    // values); otherwise the survivors' positions.
    const u64 i = dense ? p : u64(act_idx[p]);
    const u32 r2 = isa_or_zero(isa, i + 2 * h, n);
    const u32 r3 = isa_or_zero(isa, i + 3 * h, n);
    keys[p] = (u64(r2) << b) | u64(r3);
    if (!dense) vals[p] = u32(i);
  }
}

void launch_pack_quad_lo(const u32* act_idx, const SortCtl* ctl, const RoundCtl* rc, u64 n, int b,
                         const u32* isa, u64* keys, u32* vals, u32 grid, hipStream_t s) {
  hipLaunchKernelGGL(pack_quad_lo_kernel, dim3(grid), dim3(256), 0, s, act_idx, ctl, rc, n, b, isa,
                     keys, vals);
}

__global__ __launch_bounds__(256) void pack_quad_hi_kernel(const u64* __restrict__ pk,
                                                           const SortCtl* __restrict__ ctl,
                                                           const RoundCtl* __restrict__ rc, u64 n,
                                                           int b, const u32* __restrict__ isa,
                                                           u64* __restrict__ keys,
                                                           u64* __restrict__ counters) {
  const u64 count = ctl->count;
  const u64 h = rc->h;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  bool bad = false;
  for (u64 q = u64(blockIdx.x) * blockDim.x + threadIdx.x; q < count; q += stride) {
    const u64 i = u64(u32(pk[q]));
    if (i >= n) {
      bad = true;
      keys[q] = 0;
      continue;
    }
    keys[q] = (u64(isa[i]) << b) | u64(isa_or_zero(isa, i + h, n));
  }
  if (bad)
    atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
             (unsigned long long)kErrBounds);
}

void launch_pack_quad_hi(const u64* pk, const SortCtl* ctl, const RoundCtl* rc, u64 n, int b,
                         const u32* isa, u64* keys, u64* counters, u32 grid, hipStream_t s) {
  hipLaunchKernelGGL(pack_quad_hi_kernel, dim3(grid), dim3(256), 0, s, pk, ctl, rc, n, b, isa, keys,
                     counters);
}

// After the hi sort: its values are lo-sorted indices q; each becomes the
// element's position (in place) and its run name of lo goes to the other
// value buffer, which the re-rank reads as the key's tie word.
__global__ __launch_bounds__(256) void quad_permute_kernel(const SortCtl* __restrict__ ctl,
                                                           const SortPlan* __restrict__ plan,
                                                           const u64* __restrict__ pk,
                                                           u32* __restrict__ valsA,
                                                           u32* __restrict__ valsB,
                                                           u64* __restrict__ counters) {
  const u64 count = ctl->count;
  const u32 fb = plan->final_buf;
  u32* vals = fb ? valsB : valsA;
  u32* tie = fb ? valsA : valsB;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  bool bad = false;
  for (u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x; p < count; p += stride) {
    const u64 q = vals[p];
    if (q >= count) {
      bad = true;
      continue;
    }
    const u64 x = pk[q];
    vals[p] = u32(x);
    tie[p] = u32(x >> 32);
  }
  if (bad)
    atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
             (unsigned long long)kErrBounds);
}

void launch_quad_permute(const SortCtl* ctl, const SortPlan* plan, const u64* pk, u32* valsA,
                         u32* valsB, u64* counters, u32 grid, hipStream_t s) {
  hipLaunchKernelGGL(quad_permute_kernel, dim3(grid), dim3(256), 0, s, ctl, plan, pk, valsA, valsB,
                     counters);
}

// ---------------------------------------------------------------------------
// Sort control (see SortCtl): the first kernel of every sort.

__global__ __launch_bounds__(256) void sort_begin_kernel(SortCtl* __restrict__ ctl,
                                                         RoundCtl* __restrict__ rc, u64 host_count,
                                                         const u64* __restrict__ dev_count,
                                                         int npass, u64 dense_n,
                                                         int log2a,
                                                         u32* __restrict__ clear,
                                                         u64 clear_words,
                                                         u64* __restrict__ counters) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < clear_words; i += stride)
    clear[i] = 0;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  // The count is read before the counters it may come from are cleared.
  u64 count = dev_count ? *dev_count : host_count;
  // Most suffixes still active: sort them all, with keys read in order.
  const bool dense = count && dense_n && 4 * count >= 3 * dense_n;
  if (dense) count = dense_n;
  ctl->dense = dense ? 1u : 0u;
  if (rc && count) {
    const u32 k = rc->round + 1;
    if (k < u32(kMaxRounds)) {
      rc->round = k;
      rc->h = counters[kCtrChars] << (u32(log2a) * (k - 1));
      rc->active[k] = count;
      if (dense) rc->dense |= u64(1) << k;
    } else {
      atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
               (unsigned long long)kErrBounds);
      count = 0;
    }
  }
  ctl->count = count;
  ctl->gen_base = ctl->gen_next;
  ctl->gen_next = ctl->gen_next + u32(npass);
  for (int i = 0; i <= kCtrActive; ++i) counters[i] = 0;
}

void launch_sort_begin(SortCtl* ctl, RoundCtl* rc, u64 host_count, const u64* dev_count, int npass,
                       u64 dense_n, int log2a, u32* clear, u64 clear_words, u64* counters,
                       hipStream_t s) {
  u64 blocks = ceil_div(clear_words, 256 * 4);
  if (blocks < 1) blocks = 1;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(sort_begin_kernel, dim3(u32(blocks)), dim3(256), 0, s, ctl, rc, host_count,
                     dev_count, npass, dense_n, log2a, clear, clear_words, counters);
}

__global__ void sort_gen_reset_kernel(SortCtl* ctl) {
  if (threadIdx.x == 0) ctl->gen_next = 1;
}

void launch_sort_gen_reset(SortCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(sort_gen_reset_kernel, dim3(1), dim3(64), 0, s, ctl);
}

// ---------------------------------------------------------------------------
// LSD radix sort, one sweep per digit (decoupled look-back across tiles).

constexpr int kHistItems = 8;

// Up-front counts of a sort, per chunk of the input (chunk c = tiles
// [c * per, (c + 1) * per)): the digit counts of passes 0 and 1 (the
// first sweep's digit whenever one of them varies) and, over all keys, the OR
// of the keys and of their complements, which tell the plan which digits are
// constant. Later sweeps get their chunk counts from the sweep before them.
// Block b counts a contiguous share of chunk b / per_chunk.
constexpr u64 kHistBlockElems = u64(kHistBlock) * kHistItems * 4;  // a block's share, at least
constexpr u32 kHistMaxBlocks = 2048;

// Workgroups per chunk of a histogram launch of `grid` workgroups: a few per
// chunk, at most grid / nchunks. Workgroups past per * nchunks have no share.
__device__ inline u32 hist_per_chunk(const SortGeom& geo, u32 grid) {
  const u64 chunk_elems = u64(geo.tile) * geo.per;
  u64 per = (chunk_elems + kHistBlockElems - 1) / kHistBlockElems;
  const u64 cap = grid / geo.nchunks;
  if (per > cap) per = cap;
  if (per < 1) per = 1;
  return u32(per);
}

template <int RB>
__global__ __launch_bounds__(kHistBlock) void radix_histogram_kernel(
    const u64* __restrict__ keys, const SortCtl* __restrict__ ctl, u32 tile,
    u32* __restrict__ hist_in, u64* __restrict__ counters) {
  constexpr int NP = 2;
  constexpr int RADIX = 1 << RB;
  __shared__ u32 lh[NP * RADIX];
  __shared__ u64 s_or[kHistBlock / kWave], s_not[kHistBlock / kWave];
  const u64 count = ctl->count;
  if (count == 0) return;
  const SortGeom geo = sort_geom(count, tile);
  const u32 per_chunk = hist_per_chunk(geo, gridDim.x);
  if (blockIdx.x >= per_chunk * geo.nchunks) return;
  const u32 nchunks = geo.nchunks;
  const u64 chunk_elems = u64(tile) * geo.per;
  for (int i = threadIdx.x; i < NP * RADIX; i += kHistBlock) lh[i] = 0;
  __syncthreads();
  const u32 c = blockIdx.x / per_chunk;
  const u32 g = blockIdx.x % per_chunk;
  const u64 cs = u64(c) * chunk_elems;
  u64 ce = cs + chunk_elems;
  if (ce > count) ce = count;
  const int lane = lane_id();
  const u64 step = u64(kHistBlock) * kHistItems;
  u64 kor = 0, knot = 0;
  for (u64 base = cs + u64(g) * step; base < ce; base += u64(per_chunk) * step) {
    u64 key[kHistItems];
    bool valid[kHistItems];
#pragma unroll
    for (int j = 0; j < kHistItems; ++j) {
      const u64 e = base + u64(j) * kHistBlock + threadIdx.x;
      valid[j] = e < ce;
      key[j] = valid[j] ? __builtin_nontemporal_load(keys + e) : 0;
      if (valid[j]) {
        kor |= key[j];
        knot |= ~key[j];
      }
    }
#pragma unroll
    for (int j = 0; j < kHistItems; ++j) {
      const u64 vmask = __ballot(valid[j]);
      if (vmask == 0) continue;  // wave-uniform
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const u32 d = u32(key[j] >> (p * RB)) & (RADIX - 1);
        // Valid lanes form a prefix of the wave, so lane 0 is valid here.
        const u32 d0 = __shfl(d, 0, kWave);
        const u64 same = __ballot(valid[j] && d == d0);
        if (same == vmask) {
          if (lane == 0) atomicAdd(&lh[p * RADIX + d0], u32(__popcll(vmask)));
        } else if (valid[j]) {
          atomicAdd(&lh[p * RADIX + d], 1u);
        }
      }
    }
  }
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) {
    kor |= __shfl_xor(kor, off, kWave);
    knot |= __shfl_xor(knot, off, kWave);
  }
  if (lane == 0) {
    s_or[threadIdx.x / kWave] = kor;
    s_not[threadIdx.x / kWave] = knot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 o = 0, n = 0;
    for (int w = 0; w < kHistBlock / kWave; ++w) {
      o |= s_or[w];
      n |= s_not[w];
    }
    if (o) atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrKeyOr),
                    (unsigned long long)o);
    if (n) atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrKeyNot),
                    (unsigned long long)n);
  }
  if (c >= nchunks) return;
  for (int i = threadIdx.x; i < NP * RADIX; i += kHistBlock) {
    const u32 v = lh[i];
    const int p = i / RADIX, d = i % RADIX;
    if (v) atomicAdd(&hist_in[(size_t(p) * kChunks + c) * RADIX + d], v);
  }
}

// Per-chunk counts of digit plan->first_run when it is 2 or above (keys whose
// two lowest digits are constant); returns at once otherwise.
template <int RB>
__global__ __launch_bounds__(kHistBlock) void radix_histogram_first_kernel(
    const u64* __restrict__ keys, const SortCtl* __restrict__ ctl, u32 tile,
    const SortPlan* __restrict__ plan, u32* __restrict__ hist_in) {
  constexpr int RADIX = 1 << RB;
  const u64 count = ctl->count;
  if (count == 0) return;
  const u32 p = plan->first_run;
  if (p < 2) return;
  const SortGeom geo = sort_geom(count, tile);
  const u32 per_chunk = hist_per_chunk(geo, gridDim.x);
  if (blockIdx.x >= per_chunk * geo.nchunks) return;
  const u32 nchunks = geo.nchunks;
  const u64 chunk_elems = u64(tile) * geo.per;
  __shared__ u32 lh[RADIX];
  for (int i = threadIdx.x; i < RADIX; i += kHistBlock) lh[i] = 0;
  __syncthreads();
  const u32 c = blockIdx.x / per_chunk;
  const u32 g = blockIdx.x % per_chunk;
  const u64 cs = u64(c) * chunk_elems;
  u64 ce = cs + chunk_elems;
  if (ce > count) ce = count;
  const u64 step = u64(kHistBlock) * kHistItems;
  for (u64 base = cs + u64(g) * step; base < ce; base += u64(per_chunk) * step) {
#pragma unroll
    for (int j = 0; j < kHistItems; ++j) {
      const u64 e = base + u64(j) * kHistBlock + threadIdx.x;
      if (e < ce) atomicAdd(&lh[u32(keys[e] >> (p * RB)) & (RADIX - 1)], 1u);
    }
  }
  __syncthreads();
  if (c >= nchunks) return;
  for (int d = threadIdx.x; d < RADIX; d += kHistBlock) {
    const u32 v = lh[d];
    if (v) atomicAdd(&hist_in[(size_t(p) * kChunks + c) * RADIX + d], v);
  }
}

// Workgroups of a histogram launch for at most `bound` pairs: a few per chunk,
// at most kHistMaxBlocks in all (and at least kChunks, so that every chunk of
// a smaller count has one).
u32 radix_histogram_grid(u64 bound, u32 tile) {
  const SortGeom geo = sort_geom(bound, tile);
  const u64 chunk_elems = u64(tile) * geo.per;
  u64 per = ceil_div(chunk_elems, kHistBlockElems);
  const u64 cap = kHistMaxBlocks / geo.nchunks;
  if (per > cap) per = cap;
  if (per < 1) per = 1;
  u64 grid = per * geo.nchunks;
  if (grid < u64(kChunks)) grid = kChunks;
  return u32(grid);
}

void launch_radix_histogram(const u64* keys, const SortCtl* ctl, u32 tile, u32 grid,
                            u32* hist_in, u64* counters, int rb, hipStream_t s) {
#define SA_HIST(RB)                                                                          \
  hipLaunchKernelGGL(radix_histogram_kernel<RB>, dim3(grid), dim3(kHistBlock), 0, s, keys, ctl, \
                     tile, hist_in, counters)
  switch (rb) {
    case 6: SA_HIST(6); break;
    case 7: SA_HIST(7); break;
    case 9: SA_HIST(9); break;
    default: SA_HIST(8); break;
  }
#undef SA_HIST
}

void launch_radix_histogram_first(const u64* keys, const SortCtl* ctl, u32 tile, u32 grid,
                                  const SortPlan* plan, u32* hist_in, int rb, hipStream_t s) {
#define SA_HIST1(RB)                                                                        \
  hipLaunchKernelGGL(radix_histogram_first_kernel<RB>, dim3(grid), dim3(kHistBlock), 0, s, keys, \
                     ctl, tile, plan, hist_in)
  switch (rb) {
    case 6: SA_HIST1(6); break;
    case 7: SA_HIST1(7); break;
    case 9: SA_HIST1(9); break;
    default: SA_HIST1(8); break;
  }
#undef SA_HIST1
}

// The sort plan: which digits vary (the others are skipped), which buffer each
// pass reads, where values are generated and where the output ends.
__global__ void radix_plan_kernel(const SortCtl* __restrict__ ctl, const u64* __restrict__ counters,
                                  int npass, int vals_present, SortPlan* __restrict__ plan,
                                  u32* __restrict__ plan_log, int log_row,
                                  const RoundCtl* __restrict__ rc, int rb) {
  if (threadIdx.x != 0) return;
  const u64 count = ctl->count;
  if (ctl->dense) vals_present = 0;  // a dense round's values are the positions
  const u64 varying = counters[kCtrKeyOr] & counters[kCtrKeyNot];
  u32 run[kMaxPasses];
  u32 nrun = 0;
  for (int p = 0; p < kMaxPasses; ++p) {
    // (p < npass keeps the shift below 64: the passes cover at most 64 bits.)
    run[p] = (p < npass && ((varying >> (p * rb)) & ((u64(1) << rb) - 1)) != 0) ? 1u : 0u;
    nrun += run[p];
  }
  // All keys equal: one stable copy pass; nothing to sort: no pass at all.
  if (nrun == 0 && count) run[npass - 1] = 1;
  u32 cur = 0;
  bool first = true;
  int prev = -1;
  plan->first_run = 0;
  for (int p = 0; p < kMaxPasses; ++p) {
    plan->skip[p] = run[p] ? 0u : 1u;
    plan->src[p] = cur;
    plan->iota[p] = 0;
    plan->next_run[p] = -1;
    if (run[p]) {
      plan->iota[p] = (!vals_present && first) ? 1u : 0u;
      if (first) plan->first_run = u32(p);
      if (prev >= 0) plan->next_run[prev] = p;
      first = false;
      prev = p;
      cur ^= 1u;
    }
  }
  plan->final_buf = cur;
  if (!plan_log || count == 0) return;
  const int row = log_row >= 0                ? log_row
                  : log_row == kLogRowRound ? int(rc->round)
                                            : int(rc->round) + kPlanRowSecond;
  if (row >= kPlanLogRows) return;
  u32* f = plan_log + size_t(row) * kPlanLogWords;
  for (int p = 0; p < kMaxPasses; ++p) {
    f[p] = plan->skip[p];
    f[kMaxPasses + p] = plan->src[p];
    f[2 * kMaxPasses + p] = plan->iota[p];
  }
  f[3 * kMaxPasses] = cur;
}

void launch_radix_plan(const SortCtl* ctl, const u64* counters, int npass, int vals_present,
                       SortPlan* plan, u32* plan_log, int log_row, const RoundCtl* rc, int rb,
                       hipStream_t s) {
  hipLaunchKernelGGL(radix_plan_kernel, dim3(1), dim3(kWave), 0, s, ctl, counters, npass,
                     vals_present, plan, plan_log, log_row, rc, rb);
}

// One stable counting sweep over digit `pass`, persistent: workgroup b works on
// chunk b % nchunks and takes that chunk's tiles in order from a ticket. Per
// tile of BLOCK * ITEMS pairs: load ITEMS items per thread in
// wave-striped order; rank every item among the equal digits of its wave (a
// match mask of the lanes with its digit, and one LDS fetch-add per match group
// issued back to back for all items, which a wave executes in program order); combine the
// waves; publish the tile's digit counts and look back (inside the chunk) for
// the counts of earlier tiles; reorder the keys by digit in LDS and write each
// digit's run out contiguously, then the values through the same LDS buffer.
// While writing keys it counts, per output chunk, the digit of the next sweep
// that runs, so that sweep starts with exact chunk bases as well. Those counts
// are 16-bit halves in LDS: whenever the elements counted since the last check
// could carry a half past 32767 + 32767, the halves at or above 32768 move to
// the global histogram first.
// Shapes of at most 8 items per thread are held to 128 registers: 4 waves per
// SIMD, two 512-thread workgroups per CU (the 256-thread table variant, which
// LDS limits to three workgroups per CU anyway, to 168). TABLE selects how a
// wave finds the lanes that hold the same digit (see the ranking below).
template <int ITEMS, int BLOCK, bool TABLE, int RB>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(
    ITEMS <= 8 ? ((TABLE && BLOCK == 256) ? 3 : 4) : 1)))
void onesweep_pass_kernel(
    u64* __restrict__ keysA, u64* __restrict__ keysB, u32* __restrict__ valsA,
    u32* __restrict__ valsB, const SortCtl* __restrict__ ctl, int pass,
    const SortPlan* __restrict__ plan, const u32* __restrict__ hist_in,
    u32* __restrict__ hist_run, u32* __restrict__ tickets, u64* __restrict__ status,
    u64* __restrict__ counters) {
  constexpr int RADIX = 1 << RB;
  static_assert(BLOCK >= RADIX && RADIX >= kWave, "the first RADIX threads own a digit");
  constexpr int NW = BLOCK / kWave;
  constexpr int DW = RADIX / kWave;  // waves that own digits
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int kTileTz = __builtin_ctz(TILE);
  constexpr u32 kTileOdd = u32(TILE) >> kTileTz;
  __shared__ u64 s_buf[TILE];  // keys, then values (as u32)
  // Per-wave digit counts, two waves per word (16 bits each: a wave ranks at
  // most 64 * ITEMS items and a tile holds at most 6144).
  static_assert(NW % 2 == 0 && TILE < 65536, "16-bit count halves");
  __shared__ u32 s_cnt[NW / 2][RADIX];
  // With TABLE, per wave: the lanes of each digit (zero between uses).
  __shared__ u64 s_match[TABLE ? NW : 1][RADIX];
  // Next-sweep counts per (output chunk, digit), two 16-bit halves per word.
  constexpr int kNextWords = kChunks * RADIX / 2;
  constexpr u32 kNextCheck = 32768;  // elements between overflow checks
  static_assert(TILE <= int(kNextCheck), "a tile fits between two checks");
  __shared__ u32 s_next[kNextWords];
  __shared__ u32 s_start[RADIX];
  __shared__ u64 s_base[RADIX];
  __shared__ u32 s_wsum[DW];
  __shared__ u64 s_tsum[DW];
  __shared__ u32 s_ticket;
  __shared__ u32 s_abort;

  if (plan->skip[pass]) return;
  const u64 count = ctl->count;
  if (count == 0) return;
  const u32 gen = ctl->gen_base + u32(pass);
  const SortGeom geo = sort_geom(count, u32(TILE));
  const u32 nchunks = geo.nchunks;
  const u32 src = plan->src[pass];
  const bool iota = plan->iota[pass] != 0;
  const u64* kin = src ? keysB : keysA;
  u64* kout = src ? keysA : keysB;
  const u32* vin = src ? valsB : valsA;
  u32* vout = src ? valsA : valsB;
  const int shift = pass * RB;
  const int next = plan->next_run[pass];
  const int nshift = next >= 0 ? next * RB : 0;

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  const u32 chunk = blockIdx.x % nchunks;
  const u64 tiles = ceil_div(count, u64(TILE));
  const u64 c_first = u64(chunk) * geo.per;
  u64 c_end = c_first + geo.per;
  if (c_end > tiles) c_end = tiles;

  // Start of each digit's output range for this chunk: global digit offset
  // plus that digit's count in the earlier chunks.
  // Where this chunk's run of each digit starts: the digit's global start (its
  // count over all chunks, scanned over the digits) plus its count in the
  // earlier chunks.
  const bool digit_owner = tid < RADIX;  // thread tid owns digit tid
  u64 total = 0, below = 0, inc64 = 0, cbase = 0;
  if (digit_owner) {
    const u32* h = (u32(pass) == plan->first_run ? hist_in : hist_run) +
                   size_t(pass) * kChunks * RADIX;
    // Eight chunk counts in flight at a time.
    for (int c0 = 0; c0 < kChunks; c0 += 8) {
      u32 part[8];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        part[c] = u32(c0 + c) < nchunks ? h[(c0 + c) * RADIX + tid] : 0u;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        total += part[c];
        if (u32(c0 + c) < chunk) below += part[c];
      }
    }
    inc64 = wave_inclusive_sum64(total);
    if (lane == kWave - 1) s_tsum[wave] = inc64;
  }
  __syncthreads();
  if (digit_owner) {
    u64 woff = 0;
#pragma unroll
    for (int w = 0; w < DW; ++w)
      if (w < wave) woff += s_tsum[w];
    cbase = woff + inc64 - total + below;
  }
  for (int i = tid; i < kNextWords; i += BLOCK) s_next[i] = 0;
  if (TABLE)
    for (int i = tid; i < NW * RADIX; i += BLOCK) (&s_match[0][0])[i] = 0;
  u32* next_hist = hist_run + size_t(next >= 0 ? next : 0) * kChunks * RADIX;
  u32 since_check = 0;  // elements counted into s_next since every half was < 32768

  for (;;) {
    if (tid == 0) {
      s_ticket = atomicAdd(tickets + pass * kChunks + chunk, 1u);
      s_abort = 0;
    }
    for (int i = tid; i < (NW / 2) * RADIX; i += BLOCK) (&s_cnt[0][0])[i] = 0;
    if (next >= 0 && since_check + u32(TILE) > kNextCheck - 1) {
      // Every half is at most 32767 + since_check afterwards, and since_check
      // stays below 32768 until the next check: no half carries into the other.
      for (int i = tid; i < kNextWords; i += BLOCK) {
        const u32 w = s_next[i];
        u32 keep = w;
        if ((w & 0xFFFFu) >= kNextCheck) {
          atomicAdd(next_hist + 2 * i, w & 0xFFFFu);
          keep &= 0xFFFF0000u;
        }
        if ((w >> 16) >= kNextCheck) {
          atomicAdd(next_hist + 2 * i + 1, w >> 16);
          keep &= 0xFFFFu;
        }
        if (keep != w) s_next[i] = keep;
      }
      since_check = 0;
    }
    __syncthreads();
    const u64 tile = c_first + s_ticket;
    if (tile >= c_end) break;  // uniform
    const u64 tile_base = tile * TILE;
    const u64 wave_base = tile_base + u64(wave) * (ITEMS * kWave);
    // Items of this wave that exist (all of them except in the last tile).
    const u64 wleft = count > wave_base ? count - wave_base : 0;
    const u32 wvalid = wleft < u64(ITEMS * kWave) ? u32(wleft) : u32(ITEMS * kWave);
    const u64* kin_w = kin + wave_base;

    // Keys and values are both requested up front: a value load issued after
    // the key stores would wait behind them. Each input is read once per
    // sweep, so the loads are non-temporal.
    // A wave whose items all exist (every wave but those of the last tile)
    // loads without per-item tests: one address and immediate offsets.
    u64 key[ITEMS];
    u32 val[ITEMS];
    const u32* vin_w = vin + wave_base;
    if (wvalid == u32(ITEMS * kWave)) {
      const u64* kl = kin_w + lane;
      const u32* vl = vin_w + lane;
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) key[j] = __builtin_nontemporal_load(kl + j * kWave);
      if (iota) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) val[j] = u32(wave_base) + u32(j * kWave + lane);
      } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) val[j] = __builtin_nontemporal_load(vl + j * kWave);
      }
    } else {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const u32 e = u32(j * kWave + lane);
        // Missing items take the largest digit: after every valid item.
        key[j] = (e < wvalid) ? __builtin_nontemporal_load(kin_w + e) : ~u64(0);
      }
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const u32 e = u32(j * kWave + lane);
        val[j] = (e < wvalid) ? (iota ? u32(wave_base + e) : __builtin_nontemporal_load(vin_w + e))
                              : 0u;
      }
    }

    // Rank within the wave, items in (j, lane) order == input order.
    u32* cnt = &s_cnt[wave >> 1][0];
    const int half = 16 * (wave & 1);
    const u64 lt_mask = (u64(1) << lane) - 1;
    const u64 my_bit = u64(1) << lane;
    u64* mt = &s_match[TABLE ? wave : 0][0];
    u32 rank[ITEMS];
    u32 packed[ITEMS];  // below | leader << 8
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 d = digit_at<RB>(key[j], shift);
      u64 peers;
      if constexpr (TABLE) {
        // Every lane ORs its bit into the wave's table entry of its digit,
        // reads the entry back and clears it (a wave's LDS operations run in
        // order). Few vector instructions, but lanes of the same digit
        // collide in the LDS atomic unit.
        __hip_atomic_fetch_or(mt + d, my_bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        peers = mt[d];
        mt[d] = 0;
      } else {
        // Lanes whose digit differs from this lane's in some bit: the OR over
        // the bits of (ballot of the bit) XOR (this lane's bit, broadcast).
        // Each step is one three-input bitwise operation per 32-lane half
        // (diff | (ballot ^ m), truth table 0xF6). The cost does not depend on
        // the digits.
        u32 dlo = 0, dhi = 0;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          u32 m = u32(int(d << (31 - b)) >> 31);  // bit b of d in every bit
          // Opaque to the optimiser, so that the ballot compares m itself
          // instead of shifting d once more.
          asm("" : "+v"(m));
          const u64 bal = __ballot(m != 0u);
          dlo = __builtin_amdgcn_bitop3_b32(dlo, u32(bal), m, 0xF6);
          dhi = __builtin_amdgcn_bitop3_b32(dhi, u32(bal >> 32), m, 0xF6);
        }
        peers = ~(u64(dlo) | (u64(dhi) << 32));
      }
      const u32 leader = u32(__ffsll((long long)peers) - 1);
      packed[j] = u32(__popcll(peers & lt_mask)) | (leader << 8);
      u32 old = 0;
      if (u32(lane) == leader)
        old = __hip_atomic_fetch_add(cnt + d, u32(__popcll(peers)) << half, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
      rank[j] = (old >> half) & 0xFFFFu;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      rank[j] = __shfl(rank[j], int(packed[j] >> 8), kWave) + (packed[j] & 0xFFu);
    __syncthreads();

    // Per digit (one per owning thread): exclusive prefix over waves, tile
    // total.
    u32 tot = 0, inc = 0;
    if (digit_owner) {
#pragma unroll
      for (int w2 = 0; w2 < NW / 2; ++w2) {
        const u32 c = s_cnt[w2][tid];
        const u32 lo = tot, hi = tot + (c & 0xFFFFu);
        s_cnt[w2][tid] = lo | (hi << 16);
        tot = hi + (c >> 16);
      }
      u64* my_status = status + tile * RADIX + tid;
      store_status(my_status,
                   status_pack(gen, tile == c_first ? kFlagPrefix : kFlagAggregate, tot));
      // Exclusive scan of the tile totals over digits: tile-local run starts.
      inc = wave_inclusive_sum(tot);
      if (lane == kWave - 1) s_wsum[wave] = inc;
    }
    __syncthreads();
    if (digit_owner) {
      u32 woff = 0;
#pragma unroll
      for (int w = 0; w < DW; ++w)
        if (w < wave) woff += s_wsum[w];
      const u32 start = woff + inc - tot;
      s_start[tid] = start;
      // The chunk's first tile publishes a prefix, so the look-back never
      // leaves the chunk.
      u64 excl = 0;
      if (tile > c_first)
        excl = lookback(status + tid, RADIX, tile, tot, gen, false, counters, &s_abort);
      s_base[tid] = cbase + excl - u64(start);
    }
    __syncthreads();

    // Tile-local position of each item: its digit's run start, the wave's
    // offset in that run, its rank in the wave.
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 d = digit_at<RB>(key[j], shift);
      rank[j] += s_start[d] + ((s_cnt[wave >> 1][d] >> half) & 0xFFFFu);
      s_buf[rank[j]] = key[j];
    }
    __syncthreads();
    if (s_abort) return;

    const u64 left = count - tile_base;
    const u32 valid = left < u64(TILE) ? u32(left) : u32(TILE);
    since_check += valid;
    // Reordered position tid + i * BLOCK: its digit, kept for the value pass
    // (QPW digits of QB bits per register).
    constexpr int QB = RB <= 8 ? 8 : 16;
    constexpr int QPW = 32 / QB;
    u32 qdig[(ITEMS + QPW - 1) / QPW];
#pragma unroll
    for (int i = 0; i < (ITEMS + QPW - 1) / QPW; ++i) qdig[i] = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const u32 q = u32(tid + i * BLOCK);
      if (q < valid) {
        const u64 k = s_buf[q];
        const u32 d = digit_at<RB>(k, shift);
        qdig[i / QPW] |= d << (QB * (i % QPW));
        const u64 o = s_base[d] + q;
        if (o < count) {
          kout[o] = k;
          if (next >= 0) {
            // Output chunk (o / TILE) / per, with TILE = kTileOdd << kTileTz:
            // a 32-bit division by the odd factor (o < 2^(32 + kTileTz)).
            const u32 bin = chunk_of(geo, u32(o >> kTileTz) / kTileOdd) * RADIX +
                            digit_at<RB>(k, nshift);
            atomicAdd(&s_next[bin >> 1], 1u << (16 * (bin & 1u)));
          }
        }
      }
    }
    __syncthreads();
    u32* s_vals = reinterpret_cast<u32*>(s_buf);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const u32 e = u32(j * kWave + lane);
      if (e < wvalid) s_vals[rank[j]] = val[j];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const u32 q = u32(tid + i * BLOCK);
      if (q < valid) {
        const u32 d = (qdig[i / QPW] >> (QB * (i % QPW))) & ((1u << QB) - 1u);
        const u64 o = s_base[d] + q;
        if (o < count) {
          vout[o] = s_vals[q];
        } else {
          atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
                   (unsigned long long)kErrBounds);
        }
      }
    }
    __syncthreads();
  }
  if (next >= 0) {
    for (int i = tid; i < kNextWords; i += BLOCK) {
      const u32 w = s_next[i];
      if (w & 0xFFFFu) atomicAdd(next_hist + 2 * i, w & 0xFFFFu);
      if (w >> 16) atomicAdd(next_hist + 2 * i + 1, w >> 16);
    }
  }
}

bool onesweep_supported(int items, int block, bool table, int rb) {
  if (rb == kRadixBits) {
    if (block == 512) return items == 4 || items == 8 || items == 12;
    return block == 256 && (items == 8 || items == 12 || items == 16 || items == 20 ||
                            items == 24);
  }
  if (table || block != 512) return false;
  if (rb == 6 || rb == 7) return items == 4 || items == 8 || items == 12;
  if (rb == 9) return items == 8;  // 4096-pair tiles: the look-back statuses fit
  return false;
}

// Calls F with the kernel instance of a supported shape (the default shape
// otherwise).
template <typename F>
void with_onesweep(int items, int block, bool table, int rb, F&& f) {
#define SA_K(IT, BL, TB, RB) onesweep_pass_kernel<IT, BL, TB, RB>
  if (rb == 6 || rb == 7 || rb == 9) {
    if (rb == 6) {
      if (items == 4) f(SA_K(4, 512, false, 6), 512);
      else if (items == 12) f(SA_K(12, 512, false, 6), 512);
      else f(SA_K(8, 512, false, 6), 512);
    } else if (rb == 7) {
      if (items == 4) f(SA_K(4, 512, false, 7), 512);
      else if (items == 12) f(SA_K(12, 512, false, 7), 512);
      else f(SA_K(8, 512, false, 7), 512);
    } else {
      f(SA_K(8, 512, false, 9), 512);
    }
    return;
  }
  if (block == 2 * kRadix) {
    switch (items) {
      case 4: table ? f(SA_K(4, 512, true, 8), 512) : f(SA_K(4, 512, false, 8), 512); break;
      case 12: table ? f(SA_K(12, 512, true, 8), 512) : f(SA_K(12, 512, false, 8), 512); break;
      default: table ? f(SA_K(8, 512, true, 8), 512) : f(SA_K(8, 512, false, 8), 512); break;
    }
  } else {
    switch (items) {
      case 8: table ? f(SA_K(8, 256, true, 8), 256) : f(SA_K(8, 256, false, 8), 256); break;
      case 12: table ? f(SA_K(12, 256, true, 8), 256) : f(SA_K(12, 256, false, 8), 256); break;
      case 20: table ? f(SA_K(20, 256, true, 8), 256) : f(SA_K(20, 256, false, 8), 256); break;
      case 24: table ? f(SA_K(24, 256, true, 8), 256) : f(SA_K(24, 256, false, 8), 256); break;
      default: table ? f(SA_K(16, 256, true, 8), 256) : f(SA_K(16, 256, false, 8), 256); break;
    }
  }
#undef SA_K
}

void launch_onesweep_pass(u64* keysA, u64* keysB, u32* valsA, u32* valsB, const SortCtl* ctl,
                          int pass, const SortPlan* plan, const u32* hist_in, u32* hist_run,
                          u32* tickets, u64* status, u64* counters, int items, int block,
                          bool table, int rb, u32 grid, hipStream_t s) {
  with_onesweep(items, block, table, rb, [&](auto kernel, int bl) {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(bl), 0, s, keysA, keysB, valsA, valsB, ctl, pass,
                       plan, hist_in, hist_run, tickets, status, counters);
  });
}

int onesweep_wgs_per_cu(int items, int block, bool table, int rb) {
  int n = 0;
  hipError_t e = hipSuccess;
  with_onesweep(items, block, table, rb, [&](auto kernel, int bl) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, bl, 0);
  });
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

// ---------------------------------------------------------------------------
// First position q <= p whose key agrees with keys[p] in the bits above `sh`
// (x = keys[p] >> sh, sh < 64) in the ascending array `keys`: the start of the
// run (sh = 0) or group containing p. One wave, every lane: 64 probes per step,
// galloping down from p in strides 1, 64, 64^2, ... until a probe falls below
// x, then narrowing the bracketed interval 64-fold per step. A run of length L
// costs about 2 log64(L) dependent wave loads; every probe is inside [0, p].
// With TIE, elements are ordered by (key, tie[]) and the run is that of equal
// (key, tie) pairs (sh must be 0).
template <bool TIE>
__device__ u64 run_start_wave(const u64* __restrict__ keys, const u32* __restrict__ tie, u64 p,
                              int sh, u64 x, u32 tx) {
  using i64 = long long;
  const int lane = lane_id();
  auto is_below = [&](i64 pos) {
    const u64 kp = keys[pos] >> sh;
    if (!TIE) return kp < x;
    return kp < x || (kp == x && tie[pos] < tx);
  };
  i64 hi = i64(p);  // (keys[hi] >> sh) == x
  i64 lo = -1;      // (keys[lo] >> sh) < x, or -1
  i64 stride = 1;
  for (;;) {
    const i64 pos = hi - stride * (lane + 1);
    const bool below = pos < 0 || is_below(pos);
    const u64 m = __ballot(below);
    if (m) {
      const int l = __ffsll((long long)m) - 1;
      const i64 pl = hi - stride * (l + 1);
      lo = pl < -1 ? -1 : pl;
      if (l) hi -= stride * l;
      break;
    }
    hi -= stride * kWave;
    stride *= kWave;
  }
  while (hi - lo > 1) {
    const i64 st = (hi - lo + kWave - 1) / kWave;
    const i64 pos = hi - st * (lane + 1);
    const bool below = pos <= lo || is_below(pos);
    const u64 m = __ballot(below);  // lane 63 probes at or below lo: m != 0
    const int l = __ffsll((long long)m) - 1;
    const i64 nlo = hi - st * (l + 1);
    lo = nlo > lo ? nlo : lo;
    if (l) hi -= st * l;
  }
  return u64(hi);
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
// is discarded. All others survive.
//
// Layout: the tile is kRerankBlock / 64 waves of kRerankRows rows of 64
// consecutive elements; lane l of row r of wave w holds element
// base + (w * kRerankRows + r) * 64 + l, so every load and store of a row is
// one contiguous 64-element access. Within a row, the last head (group start)
// at or before each lane comes from a ballot of the head (group) flags and a
// count-leading-zeros of the bits up to the lane; the survivors' output slots
// from a population count. Rows carry the last head / group start forward;
// waves combine through LDS. No tile waits for another: the run and the group
// that the tile's first element continues from an earlier tile are found by
// searching the sorted keys (run_start_wave). Survivors collect in an LDS
// buffer of one tile's size, which takes its output range with one atomic add
// whenever it is full and once at the end, so survivors keep their sorted
// order within a workgroup's buffer but buffers land in any order (the next
// round sorts them anyway).
// TIE (quadrupling rounds): the key is (keys[p], tie word), the tie words
// being the value buffer the sort did not end in; groups still come from the
// key's upper part.
template <bool TIE>
__global__ __launch_bounds__(kRerankBlock) __attribute__((amdgpu_waves_per_eu(4)))
void rerank_compact_kernel(
    const u64* __restrict__ keysA, const u64* __restrict__ keysB,
    const u32* __restrict__ valsA, const u32* __restrict__ valsB,
    const SortPlan* __restrict__ plan, const RerankArgs a, const SortCtl* __restrict__ ctl,
    u32* __restrict__ isa, u32* __restrict__ sa_out, u32* __restrict__ act_idx,
    u64* __restrict__ act_ti, u32* __restrict__ act_rank, u64* __restrict__ counters) {
  constexpr int NW = kRerankBlock / kWave;
  constexpr int R = kRerankRows;
  constexpr int T = kRerankTile;
  static_assert(R <= 16, "flag bits of a lane: heads in 0..15, uniques in 16..31");
  const u64 count = ctl->count;
  const int mode = a.mode;
  __shared__ u32 s_wh[NW], s_wg[NW], s_ws[NW];
  __shared__ u64 s_prefix[2];
  // Survivors of the workgroup's tiles, gathered here and written out in one
  // range per buffer-full: one reservation on the shared survivor counter per
  // T survivors instead of one per tile (the atomics of all workgroups on
  // that one word serialise).
  __shared__ u64 s_sv[T];   // act_ti value (multi-text) or position
  __shared__ u32 s_svr[T];  // new name
  __shared__ u32 s_fill, s_tile_at, s_flush_n;
  __shared__ u64 s_flush_at;
  __shared__ u32 s_bh[kStageBuckets];  // staged ISA writes per position bucket

  const u32 fb = plan->final_buf;
  const u64* keys = fb ? keysB : keysA;
  const u32* vals = fb ? valsB : valsA;
  const u32* tie = fb ? valsA : valsB;  // TIE only
  const bool scatter = (mode & kRerankScatterIsa) != 0;
  const bool isa_only = (mode & kRerankIsaOnly) != 0;
  const bool pair_out = (mode & kRerankPairOut) != 0;
  const bool emit = (mode & kRerankEmit) != 0;
  const bool no_survivors = isa_only || pair_out || emit;
  const u64 emit_at = emit ? *a.emit_base : 0;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  const u64 lt_mask = (u64(1) << lane) - 1;
  const u64 tiles = ceil_div(count, u64(T));
  if (tid == 0) s_fill = 0;  // ordered before its use by the tile's first barrier
  const bool staged = scatter && a.stage_w != 0 && count >= kStageMinCount;
  u64* const stage = fb ? a.stage_a : a.stage_b;  // the key buffer the sort did not end in
  if (staged)
    for (int b = tid; b < kStageBuckets; b += kRerankBlock) s_bh[b] = 0;
  bool bad = false;
  // Writes buffer entries [0, s_flush_n) at s_flush_at (every thread).
  auto flush = [&]() {
    const u32 m = s_flush_n;
    const u64 at = s_flush_at;
    if (at + m > count) {
      bad = true;
      return;
    }
    for (u32 q = u32(tid); q < m; q += kRerankBlock) {
      const u64 w = s_sv[q];
      if (act_ti)
        act_ti[at + q] = w;
      else
        act_idx[at + q] = u32(w);
      act_rank[at + q] = s_svr[q];
    }
  };
  for (u64 tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
  const u64 base = tile * T;
  const u64 wbase = base + u64(wave) * (R * kWave);  // first element of the wave

  // The tile's elements are requested first, so that they are in flight
  // while the waves look up what precedes the tile and the text tables.
  u64 k[R];
  u32 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const u64 e = wbase + u64(r) * kWave + lane;
    k[r] = e < count ? keys[e] : 0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const u64 e = wbase + u64(r) * kWave + lane;
    v[r] = e < count ? vals[e] : 0;
  }
  u32 tw[TIE ? R : 1];
  if (TIE) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const u64 e = wbase + u64(r) * kWave + lane;
      tw[r] = e < count ? tie[e] : 0;
    }
  }

  // Multi-text: the key's top field names the text and the keys are sorted,
  // so when the wave's first and last elements lie in one text (the common
  // case: texts span many rows) its table entries serve every element of the
  // wave, loaded once instead of once per element.
  bool one_text = false;
  u64 ot = 0, ot_base = 0, ot_len = 0;
  bool ot_round0 = false;
  if (a.tbase && wbase < count) {
    const u64 wend = wbase + u64(R) * kWave;
    const u64 kf = __shfl(k[0], 0, kWave);  // keys[wbase]
    const u64 kl = wend <= count ? __shfl(k[R - 1], kWave - 1, kWave) : keys[count - 1];
    const u64 tf = kf >> a.idshift;
    if ((kl >> a.idshift) == tf) {
      one_text = true;
      ot = tf;
      ot_base = a.tbase[tf];
      ot_len = a.tlen[tf];
      ot_round0 = a.tround0[tf] != 0;
    }
  }

  // What precedes the tile: wave 0 finds the start of the run of keys equal to
  // keys[base] and wave 1 the start of its group (the last head and the last
  // group start before the tile, when the tile does not begin with one).
  if (wave < 2) {
    const u64 kb = keys[base];
    const u64 kbp = base > 0 ? keys[base - 1] : 0;
    int sh = 0;
    u64 text_start = 0;
    if (wave == 1) {
      sh = a.gshift;
      if (a.tbase) {
        // Both entries of the text at once: the start is used when the text
        // is in its round 0 (its elements form one group).
        const u64 tk = kb >> a.idshift;
        if (a.tstart) text_start = a.tstart[tk];
        if (a.tround0[tk]) sh = a.idshift;  // group = text
      }
    }
    u64 start = base;
    if (sh >= 64) {
      start = 0;  // one group holds every element
    } else if (wave == 1 && a.tstart && sh == a.idshift) {
      start = text_start;  // a round-0 text: its elements start there
    } else if (base > 0) {
      const u64 x = kb >> sh;
      if (TIE && wave == 0) {
        const u32 tb = tie[base];
        if (kbp == x && tie[base - 1] == tb)
          start = run_start_wave<true>(keys, tie, base, 0, x, tb);
      } else if ((kbp >> sh) == x) {
        start = run_start_wave<false>(keys, nullptr, base, sh, x, 0);
      }
    }
    if (lane == 0) s_prefix[wave] = start;
  }

  // Flags per element (bit r: head, bit 16 + r: unique; gflags bit r: group
  // start) and the wave's aggregates: last head, last group start (tile-local
  // position + 1, 0 = none) and survivor count.
  u32 flags = 0, gflags = 0;
  u32 wh = 0, wg = 0, ws = 0;
  const u64 edge_next = wbase + u64(R) * kWave;
  const u64 k_before = (lane == 0 && wbase > 0 && wbase - 1 < count) ? keys[wbase - 1] : 0;
  const u64 k_after = (lane == kWave - 1 && edge_next < count) ? keys[edge_next] : 0;
  u32 t_before = 0, t_after = 0;
  if (TIE) {
    t_before = (lane == 0 && wbase > 0 && wbase - 1 < count) ? tie[wbase - 1] : 0;
    t_after = (lane == kWave - 1 && edge_next < count) ? tie[edge_next] : 0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const u64 e = wbase + u64(r) * kWave + lane;
    u64 kp = __shfl_up(k[r], 1, kWave);
    u64 kn = __shfl_down(k[r], 1, kWave);
    const u64 last_prev = r > 0 ? __shfl(k[r - 1], kWave - 1, kWave) : k_before;
    const u64 first_next = r + 1 < R ? __shfl(k[r + 1], 0, kWave) : k_after;
    if (lane == 0) kp = last_prev;
    if (lane == kWave - 1) kn = first_next;
    bool diff_prev = k[r] != kp, diff_next = kn != k[r];
    if (TIE) {
      u32 tp = __shfl_up(tw[r], 1, kWave);
      u32 tn = __shfl_down(tw[r], 1, kWave);
      const u32 tl = r > 0 ? __shfl(tw[r - 1], kWave - 1, kWave) : t_before;
      const u32 tf = r + 1 < R ? __shfl(tw[r + 1], 0, kWave) : t_after;
      if (lane == 0) tp = tl;
      if (lane == kWave - 1) tn = tf;
      diff_prev = diff_prev || tw[r] != tp;
      diff_next = diff_next || tn != tw[r];
    }
    const bool valid = e < count;
    int gsh = a.gshift;
    if (valid && a.tbase && (one_text ? ot_round0 : a.tround0[k[r] >> a.idshift] != 0))
      gsh = a.idshift;  // group = text
    const bool head = valid && (e == 0 || diff_prev);
    const bool grp = valid && (e == 0 || (gsh < 64 && (k[r] >> gsh) != (kp >> gsh)));
    const bool uniq = head && (e + 1 == count || diff_next);
    // Alone in its group: its name was unique before this round, so it was
    // final already (only a dense round sorts such suffixes again).
    const bool alone = grp && (e + 1 == count || (gsh < 64 && (kn >> gsh) != (k[r] >> gsh)));
    if (head) flags |= 1u << r;
    if (uniq) flags |= 1u << (16 + r);
    if (grp) gflags |= 1u << r;
    if (alone) gflags |= 1u << (16 + r);
    const u64 hm = __ballot(head), gm = __ballot(grp), sm = __ballot(valid && !uniq);
    const u32 rowpos = u32((wave * R + r) * kWave);  // tile-local position of lane 0
    if (hm) wh = rowpos + u32(63 - __clzll((long long)hm)) + 1;
    if (gm) wg = rowpos + u32(63 - __clzll((long long)gm)) + 1;
    ws += u32(__popcll(sm));
  }
  if (lane == 0) {
    s_wh[wave] = wh;
    s_wg[wave] = wg;
    s_ws[wave] = ws;
  }
  __syncthreads();
  if (tid == 0) {
    u32 tts = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tts += s_ws[w];
    u32 fill = s_fill, fn = 0;
    if (no_survivors) tts = 0;
    if (fill + tts > u32(T)) {  // no room for this tile's survivors: empty the buffer first
      s_flush_at = atomicAdd(reinterpret_cast<unsigned long long*>(counters + kCtrActive),
                             (unsigned long long)fill);
      fn = fill;
      fill = 0;
    }
    s_flush_n = fn;
    s_tile_at = fill;
    s_fill = fill + tts;
  }
  __syncthreads();
  if (s_flush_n) {
    flush();
    __syncthreads();  // the buffer is refilled below
  }

  // Carries into the wave's first row: from earlier waves of the tile, else
  // from before the tile.
  u32 eh = 0, eg = 0, es = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wave) {
      eh = s_wh[w] > eh ? s_wh[w] : eh;
      eg = s_wg[w] > eg ? s_wg[w] : eg;
      es += s_ws[w];
    }
  }
  u64 carry_h = eh ? base + eh - 1 : s_prefix[0];
  u64 carry_g = eg ? base + eg - 1 : s_prefix[1];
  u32 out_base = s_tile_at + es;  // buffer slot of the wave's first survivor
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const u64 e = wbase + u64(r) * kWave + lane;
    const u64 row0 = wbase + u64(r) * kWave;
    const bool head = (flags >> r) & 1u;
    const bool uniq = (flags >> (16 + r)) & 1u;
    const bool grp = (gflags >> r) & 1u;
    const bool valid = e < count;
    const u64 hm = __ballot(head), gm = __ballot(grp), sm = __ballot(valid && !uniq);
    const u64 upto = lt_mask | (u64(1) << lane);
    const u64 hmine = hm & upto, gmine = gm & upto;
    const u64 ss = hmine ? row0 + u64(63 - __clzll((long long)hmine)) : carry_h;
    const u64 gs = gmine ? row0 + u64(63 - __clzll((long long)gmine)) : carry_g;
    const u32 out = out_base + u32(__popcll(sm & lt_mask));
    if (hm) carry_h = row0 + u64(63 - __clzll((long long)hm));
    if (gm) carry_g = row0 + u64(63 - __clzll((long long)gm));
    out_base += u32(__popcll(sm));
    if (!valid) continue;
    // Text of the element: the whole text, or (multi-text) the one named by
    // the key's high bits; ranks and positions are local to it.
    u64 gb = 0, nt = a.n, t = 0;
    bool first_round = a.rmask == 0;
    if (one_text) {
      t = ot;
      gb = ot_base;
      nt = ot_len;
      first_round = ot_round0;
    } else if (a.tbase) {
      t = k[r] >> a.idshift;
      gb = a.tbase[t];
      nt = a.tlen[t];
      first_round = a.tround0[t] != 0;
    }
    const u64 r0 = first_round ? 1 : ((k[r] >> a.rshift) & a.rmask);
    const u64 nr = r0 + ss - gs;
    if (v[r] >= nt || nr == 0 || nr > nt || (!uniq && !no_survivors && out >= u32(T))) {
      bad = true;
      if (staged) stage[e] = kStageSkip;
      continue;
    }
    if (pair_out) {
      a.pair_out[e] = (nr << 32) | u64(v[r]);
      continue;
    }
    if (emit) {
      a.emit_keys[emit_at + e] = opk_key(v[r], a.emit_h, a.emit_q) | (uniq ? kUniqueBit : 0);
      a.emit_vals[emit_at + e] = u32(nr);
      continue;
    }
    // The ISA already holds every active suffix's previous name, so a name
    // that did not change (a group that did not split, or the first sub-group
    // of one that did) is not written again.
    if (staged) {
      u64 w = kStageSkip;
      if (first_round || nr != r0) {
        const u32 pos = u32(gb + v[r]);
        w = (u64(pos) << 32) | u64(u32(nr));
        atomicAdd(&s_bh[pos / a.stage_w], 1u);
      }
      stage[e] = w;
    } else if (scatter && (first_round || nr != r0)) {
      isa[gb + v[r]] = u32(nr);
    }
    if (isa_only) continue;
    if (uniq) {
      if (first_round || !((gflags >> (16 + r)) & 1u)) sa_out[gb + nr - 1] = v[r];
    } else {
      s_sv[out] = act_ti ? ((t << 32) | v[r]) : u64(v[r]);
      s_svr[out] = u32(nr);
    }
  }
  __syncthreads();  // the next tile reuses the LDS aggregates
  }
  // The survivors still in the buffer.
  if (tid == 0) {
    const u32 fill = s_fill;
    s_flush_n = fill;
    if (fill)
      s_flush_at = atomicAdd(reinterpret_cast<unsigned long long*>(counters + kCtrActive),
                             (unsigned long long)fill);
  }
  __syncthreads();
  if (s_flush_n) flush();
  if (staged)
    for (int b = tid; b < kStageBuckets; b += kRerankBlock)
      a.stage_hist[size_t(b) * gridDim.x + blockIdx.x] = s_bh[b];
  if (bad)
    atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
             (unsigned long long)kErrBounds);
}

int rerank_wgs_per_cu(bool tie) {
  static std::atomic<int> cache[2];
  int n = cache[tie ? 1 : 0].load(std::memory_order_relaxed);
  if (n > 0) return n;
  const hipError_t e =
      tie ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rerank_compact_kernel<true>,
                                                         kRerankBlock, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rerank_compact_kernel<false>,
                                                         kRerankBlock, 0);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return 4;
  }
  cache[tie ? 1 : 0].store(n, std::memory_order_relaxed);
  return n;
}

void launch_rerank_compact(const u64* keysA, const u64* keysB, const u32* valsA,
                           const u32* valsB, const SortPlan* plan, const RerankArgs& args,
                           const SortCtl* ctl, u32* isa, u32* sa_out, u32* act_idx, u64* act_ti,
                           u32* act_rank, u64* counters, u32 grid, hipStream_t s) {
  if (args.tie)
    hipLaunchKernelGGL(rerank_compact_kernel<true>, dim3(grid), dim3(kRerankBlock), 0, s, keysA,
                       keysB, valsA, valsB, plan, args, ctl, isa, sa_out, act_idx, act_ti, act_rank,
                       counters);
  else
    hipLaunchKernelGGL(rerank_compact_kernel<false>, dim3(grid), dim3(kRerankBlock), 0, s, keysA,
                       keysB, valsA, valsB, plan, args, ctl, isa, sa_out, act_idx, act_ti, act_rank,
                       counters);
}

// ---------------------------------------------------------------------------
// Staged ISA writes of a re-rank (see RerankArgs::stage_w). A random 4-byte
// write costs a memory transaction of its own; with the pairs grouped by
// position bucket, the writes a wave of the last kernel issues fall in one
// 1/kStageBuckets stretch of the ISA, whose lines the caches then combine.

// Exclusive scan, in place, of the per-(bucket, workgroup) counts in
// bucket-major order (one workgroup); the total to counters[kCtrStage].
__global__ __launch_bounds__(1024) void stage_scan_kernel(const SortCtl* __restrict__ ctl,
                                                          u32* __restrict__ hist, u32 entries,
                                                          u64* __restrict__ counters) {
  if (ctl->count < kStageMinCount) return;
  __shared__ u32 s_w[1024 / kWave];
  const u32 tid = threadIdx.x;
  const u32 per = (entries + 1023) / 1024;
  const u32 lo = tid * per < entries ? tid * per : entries;
  const u32 hi = lo + per < entries ? lo + per : entries;
  u32 sum = 0;
  for (u32 i = lo; i < hi; ++i) sum += hist[i];
  const u32 inc = wave_inclusive_sum(sum);
  if (lane_id() == kWave - 1) s_w[tid / kWave] = inc;
  __syncthreads();
  u32 run = inc - sum;
  for (u32 w = 0; w < tid / kWave; ++w) run += s_w[w];
  for (u32 i = lo; i < hi; ++i) {
    const u32 x = hist[i];
    hist[i] = run;
    run += x;
  }
  if (tid == 1023) counters[kCtrStage] = run;
}

// Each workgroup takes the tiles its re-rank workgroup took (same grid, same
// tile order) and moves their staged pairs to the scanned offsets of their
// buckets in the key buffer the sort ended in.
__global__ __launch_bounds__(256) void stage_partition_kernel(
    u64* __restrict__ keysA, u64* __restrict__ keysB, const SortPlan* __restrict__ plan,
    const SortCtl* __restrict__ ctl, const u32* __restrict__ hist, u32 stage_w, u64 n,
    u64* __restrict__ counters) {
  constexpr int T = kRerankTile;
  constexpr int PER = T / 256;
  const u64 count = ctl->count;
  if (count < kStageMinCount) return;
  const u32 fb = plan->final_buf;
  const u64* stage = fb ? keysA : keysB;
  u64* out = fb ? keysB : keysA;
  __shared__ u32 s_off[kStageBuckets], s_cnt[kStageBuckets];
  const int tid = threadIdx.x;
  for (int b = tid; b < kStageBuckets; b += 256) {
    s_off[b] = hist[size_t(b) * gridDim.x + blockIdx.x];
    s_cnt[b] = 0;
  }
  __syncthreads();
  const u64 total = counters[kCtrStage];
  const u64 tiles = ceil_div(count, u64(T));
  bool bad = false;
  for (u64 tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    u64 w[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const u64 e = tile * T + u64(j) * 256 + tid;
      w[j] = e < count ? stage[e] : kStageSkip;
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (w[j] == kStageSkip) continue;
      const u64 pos = w[j] >> 32;
      if (pos >= n) {
        bad = true;
        continue;
      }
      const u32 b = u32(pos) / stage_w;  // < kStageBuckets: stage_w >= n / kStageBuckets
      const u64 slot = u64(s_off[b]) + atomicAdd(&s_cnt[b], 1u);
      if (slot >= total) {
        bad = true;
        continue;
      }
      out[slot] = w[j];
    }
    __syncthreads();
    for (int b = tid; b < kStageBuckets; b += 256) {
      s_off[b] += s_cnt[b];
      s_cnt[b] = 0;
    }
    __syncthreads();
  }
  if (bad)
    atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
             (unsigned long long)kErrBounds);
}

// ISA[position] = name for the grouped pairs, in order: the threads in flight
// write into one or two buckets' stretches. Scattered 4-byte writes run
// fastest with few in flight: about four 256-thread workgroups per CU (twice
// as many take twice as long).
__global__ __launch_bounds__(256) void stage_apply_kernel(const u64* __restrict__ keysA,
                                                          const u64* __restrict__ keysB,
                                                          const SortPlan* __restrict__ plan,
                                                          const SortCtl* __restrict__ ctl,
                                                          const u64* __restrict__ counters, u64 n,
                                                          u32* __restrict__ isa) {
  if (ctl->count < kStageMinCount) return;
  const u64* in = plan->final_buf ? keysB : keysA;
  const u64 total = counters[kCtrStage];
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 e = u64(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const u64 w = in[e];
    const u64 pos = w >> 32;
    if (pos < n) isa[pos] = u32(w);
  }
}

void launch_stage_isa(u64* keysA, u64* keysB, const SortPlan* plan, const SortCtl* ctl,
                      u32* stage_hist, u32 grid, u32 stage_w, u64 n, u32* isa, u64* counters,
                      u32 apply_grid, hipStream_t s) {
  hipLaunchKernelGGL(stage_scan_kernel, dim3(1), dim3(1024), 0, s, ctl, stage_hist,
                     u32(kStageBuckets) * grid, counters);
  hipLaunchKernelGGL(stage_partition_kernel, dim3(grid), dim3(256), 0, s, keysA, keysB, plan, ctl,
                     stage_hist, stage_w, n, counters);
  hipLaunchKernelGGL(stage_apply_kernel, dim3(apply_grid), dim3(256), 0, s, keysA, keysB, plan,
                     ctl, counters, n, isa);
}

// ---------------------------------------------------------------------------
// Inverse suffix array after round 0.
//
// Eager form: ISA[text position] = rank for every sorted position (one random
// 4-byte write per suffix), written by a second pass of the round-0 re-rank.
// Round 0 itself writes no ISA, so that the lazy form, used when few suffixes
// survive round 0, pays for no rank array either:
// only the survivors' ranks are written and marked in a bitmap of live
// positions; a later gather of an unmarked position j recomputes its round-0
// rank as 1 + the number of round-0 keys below key(j), by binary search in the
// round-0 sorted keys (the name is the head rank of j's run of equal keys).

__global__ __launch_bounds__(256) void isa_scatter_list_kernel(const u32* __restrict__ idx,
                                                               const u32* __restrict__ rank,
                                                               u64 count, u64 n,
                                                               u32* __restrict__ isa,
                                                               u32* __restrict__ live) {
  u64 q = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const u32 v = idx[q];
  if (v < n) {
    isa[v] = rank[q];
    atomicOr(&live[v >> 5], 1u << (v & 31u));
  }
}

void launch_isa_scatter_list(const u32* idx, const u32* rank, u64 count, u64 n, u32* isa,
                             u32* live, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(isa_scatter_list_kernel, dim3(u32(ceil_div(count, 256))), dim3(256), 0, s,
                     idx, rank, count, n, isa, live);
}

namespace {

// Round-0 name of suffix j: its packed key and a lower-bound search in the
// round-0 sorted keys. The search starts in `sample` (kLazySamples keys of the
// sorted array, sample[i] = keys0[i * n / kLazySamples], staged in LDS), which
// narrows it to a range of n / kLazySamples keys before the global steps.
__device__ inline u32 round0_rank(u64 j, const u8* __restrict__ text, u64 n,
                                  const u16* __restrict__ code, u32 w, u32 c,
                                  const u64* __restrict__ keys0, const u64* __restrict__ sample) {
  u64 k = 0;
  for (u32 q = 0; q < c; ++q) {
    const u64 p = j + q;
    k = (k << w) | u64(p < n ? code[text[p]] : u16(0));
  }
  // First sample not below k.
  u32 slo = 0, shi = kLazySamples;
  while (slo < shi) {
    const u32 mid = (slo + shi) >> 1;
    if (sample[mid] < k)
      slo = mid + 1;
    else
      shi = mid;
  }
  // keys0[pos(slo - 1)] < k <= keys0[pos(slo)]: the lower bound lies between.
  u64 lo = slo ? (u64(slo - 1) * n) / kLazySamples + 1 : 0;
  u64 hi = slo < kLazySamples ? (u64(slo) * n) / kLazySamples : n;
  while (lo < hi) {
    const u64 mid = (lo + hi) >> 1;
    if (keys0[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return u32(lo + 1);
}

}  // namespace

__global__ __launch_bounds__(256) void lazy_sample_kernel(const u64* __restrict__ keys0, u64 n,
                                                          u64* __restrict__ sample) {
  const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kLazySamples) sample[i] = keys0[(u64(i) * n) / kLazySamples];
}

void launch_lazy_sample(const u64* keys0, u64 n, u64* sample, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(lazy_sample_kernel, dim3(kLazySamples / 256), dim3(256), 0, s, keys0, n,
                     sample);
}

// A persistent grid: each workgroup stages the code table and the sample in
// LDS once and strides over the active suffixes.
__global__ __launch_bounds__(256) void pack_pairs_lazy_kernel(
    const u32* __restrict__ act_idx, const u32* __restrict__ act_rank,
    const SortCtl* __restrict__ ctl, const RoundCtl* __restrict__ rc, u64 n, int b,
    const u32* __restrict__ isa, const u8* __restrict__ text, const u16* __restrict__ code,
    const u64* __restrict__ counters, const u64* __restrict__ keys0,
    const u64* __restrict__ sample, const u32* __restrict__ live, u64* __restrict__ keys,
    u32* __restrict__ vals) {
  __shared__ u16 s_code[256];
  __shared__ u64 s_sample[kLazySamples];
  const u64 count = ctl->count;
  if (u64(blockIdx.x) * blockDim.x >= count) return;
  s_code[threadIdx.x] = code[threadIdx.x];
  for (u32 i = threadIdx.x; i < kLazySamples; i += 256) s_sample[i] = sample[i];
  __syncthreads();
  const u64 h = rc->h;
  const u32 w = u32(counters[kCtrCodeBits]);
  const u32 c = u32(counters[kCtrChars]);
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x; p < count; p += stride) {
    const u32 i = act_idx[p];
    const u32 r = act_rank[p];
    const u64 j = u64(i) + h;
    u32 r1 = 0;
    if (j < n) {
      // ISA[j] holds a name only for suffixes that survived round 0.
      if ((live[j >> 5] >> (j & 31u)) & 1u)
        r1 = isa[j];
      else
        r1 = round0_rank(j, text, n, s_code, w, c, keys0, s_sample);
    }
    keys[p] = (u64(r) << b) | u64(r1);
    vals[p] = i;
  }
}

void launch_pack_pairs_lazy(const u32* act_idx, const u32* act_rank, const SortCtl* ctl,
                            const RoundCtl* rc, u64 n, int b, const u32* isa, const u8* text,
                            const u16* code, const u64* counters, const u64* keys0,
                            const u64* sample, const u32* live, u64* keys, u32* vals, u32 grid,
                            hipStream_t s) {
  hipLaunchKernelGGL(pack_pairs_lazy_kernel, dim3(grid), dim3(256), 0, s, act_idx, act_rank, ctl,
                     rc, n, b, isa, text, code, counters, keys0, sample, live, keys, vals);
}

__global__ __launch_bounds__(256) void isa_complete_kernel(u32* __restrict__ isa, u64 n,
                                                           const u8* __restrict__ text,
                                                           const u16* __restrict__ code,
                                                           const u64* __restrict__ counters,
                                                           const u64* __restrict__ keys0,
                                                           const u64* __restrict__ sample,
                                                           const u32* __restrict__ live) {
  __shared__ u16 s_code[256];
  __shared__ u64 s_sample[kLazySamples];
  s_code[threadIdx.x] = code[threadIdx.x];
  for (u32 i = threadIdx.x; i < kLazySamples; i += 256) s_sample[i] = sample[i];
  __syncthreads();
  u64 j = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if ((live[j >> 5] >> (j & 31u)) & 1u) return;
  const u32 w = u32(counters[kCtrCodeBits]);
  const u32 c = u32(counters[kCtrChars]);
  isa[j] = round0_rank(j, text, n, s_code, w, c, keys0, s_sample);
}

void launch_isa_complete(u32* isa, u64 n, const u8* text, const u16* code, const u64* counters,
                         const u64* keys0, const u64* sample, const u32* live, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(isa_complete_kernel, dim3(u32(ceil_div(n, 256))), dim3(256), 0, s, isa, n,
                     text, code, counters, keys0, sample, live);
}

// ---------------------------------------------------------------------------
// Multi-text engine: many texts in one round. Keys carry the text slot in their
// high bits so that one sort and one re-rank per round serve every text; each
// text has its own alphabet codes, its own round and its own doubling offset.

namespace {

// Index i of the new text owning chunk `b`: the last i with chunk0[i] <= b.
__device__ inline u32 new_text_of(const u64* __restrict__ chunk0, u32 m, u64 b) {
  u32 lo = 0, hi = m;
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (chunk0[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

}  // namespace

// Each workgroup scans a contiguous range of chunks (chunks of one text are
// consecutive), marking the bytes seen in an LDS table and flushing it into
// the text's bitmap whenever the text changes.
__global__ __launch_bounds__(256) void multi_presence_kernel(const u8* __restrict__ arena,
                                                             TextTab tab, NewList nl,
                                                             u64 per_block) {
  __shared__ u32 seen[256];
  const u64 b0 = u64(blockIdx.x) * per_block;
  u64 b1 = b0 + per_block;
  if (b1 > nl.chunks) b1 = nl.chunks;
  if (b0 >= b1) return;
  u32 i = new_text_of(nl.chunk0, nl.m, b0);
  u64 b = b0;
  while (b < b1) {
    while (i + 1 < nl.m && nl.chunk0[i + 1] <= b) ++i;
    const u32 t = nl.t[i];
    const u64 bend = (nl.chunk0[i + 1] < b1) ? nl.chunk0[i + 1] : b1;  // this text's chunks
    seen[threadIdx.x] = 0;
    __syncthreads();
    const u64 len = tab.len[t];
    const u64 start = (b - nl.chunk0[i]) * kNewChunk;
    u64 end = (bend - nl.chunk0[i]) * kNewChunk;
    if (end > len) end = len;
    // Absolute byte range: 16-byte words inside, single bytes at the ends.
    const u64 lo = tab.base[t] + start, hi = tab.base[t] + end;
    u64 alo = (lo + 15) & ~u64(15), ahi = hi & ~u64(15);
    if (alo > ahi) alo = ahi = hi;
    const uint4* v = reinterpret_cast<const uint4*>(arena + alo);
    const u64 words = (ahi - alo) / 16;
    for (u64 q = threadIdx.x; q < words; q += 256) {
      const uint4 w = v[q];
      const u32 ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int by = 0; by < 4; ++by) seen[(ws[k] >> (8 * by)) & 0xFFu] = 1;
      }
    }
    for (u64 q = lo + threadIdx.x; q < alo; q += 256) seen[arena[q]] = 1;
    for (u64 q = ahi + threadIdx.x; q < hi; q += 256) seen[arena[q]] = 1;
    __syncthreads();
    // One atomic per 32 byte values: many workgroups flush into the same
    // eight words of a long text.
    const u64 m = __ballot(seen[threadIdx.x] != 0);
    const int lane = lane_id();
    if (lane == 0 || lane == 32) {
      const u32 bits = u32(m >> lane);
      if (bits) atomicOr(&tab.present[t * 8 + threadIdx.x / 32], bits);
    }
    __syncthreads();
    b = bend;
  }
}

void launch_multi_presence(const u8* arena, TextTab tab, NewList nl, hipStream_t s) {
  if (nl.chunks == 0) return;
  u64 blocks = nl.chunks < 2048 ? nl.chunks : 2048;
  const u64 per = ceil_div(nl.chunks, blocks);
  blocks = ceil_div(nl.chunks, per);
  hipLaunchKernelGGL(multi_presence_kernel, dim3(u32(blocks)), dim3(256), 0, s, arena, tab, nl,
                     per);
}

// Code table and characters per key of each joining text. The characters take
// at most `avail_bits` key bits (below the text id's idbits); with `trim` the
// count is then cut to end on a radix digit boundary.
__global__ __launch_bounds__(256) void multi_codes_kernel(TextTab tab, NewList nl, int idbits,
                                                          int avail_bits, int trim, int rb) {
  __shared__ u32 wsum[4];
  const u32 t = nl.t[blockIdx.x];
  const int d = threadIdx.x;
  const u32 p = (tab.present[t * 8 + d / 32] >> (d % 32)) & 1u;
  const u32 inc = wave_inclusive_sum(p);
  if (lane_id() == kWave - 1) wsum[d / kWave] = inc;
  __syncthreads();
  u32 off = 0, total = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < d / kWave) off += wsum[w];
    total += wsum[w];
  }
  tab.code[size_t(t) * 256 + d] = p ? u16(off + inc) : u16(0);
  __syncthreads();
  if (d < 8) tab.present[t * 8 + d] = 0;  // clean for the slot's next text
  if (d == 0) {
    u32 w = 32 - __clz(total);
    if (w == 0) w = 1;
    const u32 avail = u32(avail_bits);
    u32 c = avail / w;
    if (c < 1) c = 1;
    const u32 used = u32(idbits) + c * w;
    const u32 urb = u32(rb);
    if (trim && used % urb != 0 && used > urb) {
      const u32 full = (used / urb) * urb;
      if (full > u32(idbits)) {
        const u32 ct = (full - u32(idbits)) / w;
        if (ct >= 1) c = ct;
      }
    }
    // A key that reaches the last digit of 64 bits costs one sweep more; drop
    // characters to one digit fewer while at least 12 remain (an alphabet of
    // at most 7 symbols).
    const u32 fewer = u32(passes_for(64, rb) - 1) * urb;
    if (trim && u32(idbits) + c * w > fewer && fewer > u32(idbits)) {
      const u32 ct = (fewer - u32(idbits)) / w;
      if (ct >= 12) c = ct;
    }
    tab.wc[t] = w | (c << 16);
  }
}

void launch_multi_codes(TextTab tab, NewList nl, int idbits, int avail_bits, int trim, int rb,
                        hipStream_t s) {
  if (nl.m == 0) return;
  hipLaunchKernelGGL(multi_codes_kernel, dim3(nl.m), dim3(256), 0, s, tab, nl, idbits, avail_bits,
                     trim, rb);
}

__global__ __launch_bounds__(kPackBlock) void multi_pack0_kernel(const u8* __restrict__ arena,
                                                                 TextTab tab, NewList nl,
                                                                 int idshift,
                                                                 u64* __restrict__ keys,
                                                                 u32* __restrict__ vals) {
  static_assert(kNewChunk == kPackTile, "one chunk per packing workgroup");
  __shared__ u16 s_code[256];
  __shared__ u16 s_sym[kPackTile + kPackHalo];
  __shared__ u64 s_out[kPackBlock * (kPackItems + 1)];
  const int th = threadIdx.x;
  const u64 b = blockIdx.x;
  const u32 i = new_text_of(nl.chunk0, nl.m, b);
  const u32 t = nl.t[i];
  const u64 start = (b - nl.chunk0[i]) * kNewChunk;
  const u64 len = tab.len[t];
  const u8* txt = arena + tab.base[t];
  const u32 wc = tab.wc[t];
  const u32 w = wc & 0xFFFFu, c = wc >> 16;
  s_code[th] = tab.code[size_t(t) * 256 + th];
  __syncthreads();
  for (int q = th; q < kPackTile + kPackHalo; q += kPackBlock) {
    const u64 p = start + u64(q);
    s_sym[q] = (p < len) ? s_code[txt[p]] : u16(0);
  }
  __syncthreads();
  const u64 keymask = (c * w >= 64) ? ~u64(0) : ((u64(1) << (c * w)) - 1);
  const int first = th * kPackItems;
  u64 key = 0;
  for (u32 j = 0; j < c; ++j) key = (key << w) | u64(s_sym[first + int(j)]);
  s_out[pad_out<kPackItems>(th, 0)] = key;
#pragma unroll
  for (int j = 1; j < kPackItems; ++j) {
    key = ((key << w) | u64(s_sym[first + j + int(c) - 1])) & keymask;
    s_out[pad_out<kPackItems>(th, j)] = key;
  }
  __syncthreads();
  const u64 tag = u64(t) << idshift;
  const u64 out = nl.out[i] + start;
  for (int q = th; q < kPackTile; q += kPackBlock) {
    const u64 p = start + u64(q);
    if (p < len) {
      __builtin_nontemporal_store(tag | s_out[pad_out<kPackItems>(q / kPackItems, q % kPackItems)],
                                  keys + out + q);
      __builtin_nontemporal_store(u32(p), vals + out + q);
    }
  }
}

void launch_multi_pack0(const u8* arena, TextTab tab, NewList nl, int idshift, u64* keys,
                        u32* vals, hipStream_t s) {
  if (nl.chunks == 0) return;
  hipLaunchKernelGGL(multi_pack0_kernel, dim3(u32(nl.chunks)), dim3(kPackBlock), 0, s, arena, tab,
                     nl, idshift, keys, vals);
}

__global__ __launch_bounds__(256) void multi_pack_pairs_kernel(
    const u64* __restrict__ act_ti, const u32* __restrict__ act_rank, u64 count, TextTab tab,
    int b, int idshift, const u32* __restrict__ isa, u64* __restrict__ keys,
    u32* __restrict__ vals) {
  const u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const u64 ti = act_ti[p];
  const u64 t = ti >> 32;
  const u32 i = u32(ti);
  const u64 gb = tab.base[t];
  const u64 nt = tab.len[t];
  const u64 j = u64(i) + tab.h[t];
  const u32 r1 = (j < nt) ? isa[gb + j] : 0u;
  keys[p] = (t << idshift) | (u64(act_rank[p]) << b) | u64(r1);
  vals[p] = i;
}

void launch_multi_pack_pairs(const u64* act_ti, const u32* act_rank, u64 count, TextTab tab,
                             int b, int idshift, const u32* isa, u64* keys, u32* vals,
                             hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(multi_pack_pairs_kernel, dim3(u32(ceil_div(count, 256))), dim3(256), 0, s,
                     act_ti, act_rank, count, tab, b, idshift, isa, keys, vals);
}

// Batched build, lazy ISA after round 0 (as for one text): only the
// survivors' names are scattered and marked live; a gather of an unmarked
// position recomputes its round-0 name by a lower-bound search for its key in
// the text's own range of the round-0 sorted keys, which is contiguous because
// the text slot leads every key.
__global__ __launch_bounds__(256) void multi_isa_scatter_list_kernel(
    const u64* __restrict__ act_ti, const u32* __restrict__ act_rank,
    const u64* __restrict__ count_ptr, TextTab tab, u32* __restrict__ isa,
    u32* __restrict__ live) {
  const u64 count = *count_ptr;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x; p < count; p += stride) {
    const u64 ti = act_ti[p];
    const u64 t = ti >> 32;
    const u64 v = u32(ti);
    if (v >= tab.len[t]) continue;
    const u64 g = tab.base[t] + v;
    isa[g] = act_rank[p];
    atomicOr(&live[g >> 5], 1u << (g & 31u));
  }
}

void launch_multi_isa_scatter_list(const u64* act_ti, const u32* act_rank, const u64* count_ptr,
                                   u64 bound, TextTab tab, u32* isa, u32* live, hipStream_t s) {
  if (bound == 0) return;
  u64 blocks = ceil_div(bound, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(multi_isa_scatter_list_kernel, dim3(u32(blocks)), dim3(256), 0, s, act_ti,
                     act_rank, count_ptr, tab, isa, live);
}

__global__ __launch_bounds__(256) void multi_pack_pairs_lazy_kernel(
    const u64* __restrict__ act_ti, const u32* __restrict__ act_rank, u64 count, TextTab tab,
    int b, int idshift, int idshift0, const u32* __restrict__ isa, const u32* __restrict__ live,
    const u8* __restrict__ arena, const u64* __restrict__ keys0, u64* __restrict__ keys,
    u32* __restrict__ vals) {
  const u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const u64 ti = act_ti[p];
  const u64 t = ti >> 32;
  const u32 i = u32(ti);
  const u64 gb = tab.base[t];
  const u64 nt = tab.len[t];
  const u64 j = u64(i) + tab.h[t];
  u32 r1 = 0;
  if (j < nt) {
    const u64 g = gb + j;
    if ((live[g >> 5] >> (g & 31u)) & 1u) {
      r1 = isa[g];
    } else {
      // The text's round-0 key of position j, then its lower bound among the
      // text's sorted round-0 keys.
      const u32 wc = tab.wc[t];
      const u32 w = wc & 0xFFFFu, c = wc >> 16;
      const u16* code = tab.code + size_t(t) * 256;
      const u8* txt = arena + gb;
      u64 k = 0;
      for (u32 q = 0; q < c; ++q) {
        const u64 pos = j + q;
        k = (k << w) | u64(pos < nt ? code[txt[pos]] : u16(0));
      }
      k |= t << idshift0;  // the round-0 keys' layout
      u64 lo = gb, hi = gb + nt;
      while (lo < hi) {
        const u64 mid = (lo + hi) >> 1;
        if (keys0[mid] < k)
          lo = mid + 1;
        else
          hi = mid;
      }
      r1 = u32(lo - gb + 1);
    }
  }
  keys[p] = (t << idshift) | (u64(act_rank[p]) << b) | u64(r1);
  vals[p] = i;
}

void launch_multi_pack_pairs_lazy(const u64* act_ti, const u32* act_rank, u64 count, TextTab tab,
                                  int b, int idshift, int idshift0, const u32* isa,
                                  const u32* live, const u8* arena, const u64* keys0, u64* keys,
                                  u32* vals, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(multi_pack_pairs_lazy_kernel, dim3(u32(ceil_div(count, 256))), dim3(256), 0,
                     s, act_ti, act_rank, count, tab, b, idshift, idshift0, isa, live, arena,
                     keys0, keys, vals);
}

__global__ __launch_bounds__(256) void multi_count_survivors_kernel(
    const u64* __restrict__ act_ti, const u64* __restrict__ count_ptr, u32* __restrict__ surv) {
  const u64 count = *count_ptr;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  // Grid-stride with a wave-uniform trip count so that every lane takes part
  // in the shuffles and ballots.
  for (u64 base = u64(blockIdx.x) * blockDim.x; base < count; base += stride) {
    const u64 p = base + threadIdx.x;
    const bool valid = p < count;
    const u32 t = valid ? u32(act_ti[p] >> 32) : 0xFFFFFFFFu;
    // Survivors of one text are mostly adjacent: one atomic per run in the wave.
    const u32 tprev = __shfl_up(t, 1, kWave);
    const bool lead = valid && (lane_id() == 0 || tprev != t);
    const u64 leads = __ballot(lead);
    const u64 vm = __ballot(valid);
    if (lead) {
      const u64 above = leads & ~((u64(2) << lane_id()) - 1);  // next run start in the wave
      const int next = above ? __ffsll((long long)above) - 1 : kWave;
      const int last_valid = 63 - __clzll((long long)vm);
      const int end = next < kWave ? next : last_valid + 1;
      atomicAdd(&surv[t], u32(end - lane_id()));
    }
  }
}

void launch_multi_count_survivors(const u64* act_ti, const u64* count_ptr, u64 bound, u32* surv,
                                  hipStream_t s) {
  if (bound == 0) return;
  u64 blocks = ceil_div(bound, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(multi_count_survivors_kernel, dim3(u32(blocks)), dim3(256), 0, s, act_ti,
                     count_ptr, surv);
}

}  // namespace sa
