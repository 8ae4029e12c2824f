// Index structures computed on the GPU from a text and its suffix array, the
// step the paper's conclusion names after suffix sorting: the LCP array, the
// Burrows-Wheeler transform of text$, and an FM index that answers pattern
// queries by backward search over the transform.
//
// LCP array, in two parts. First, in suffix array order, LCP[j] is found by
// comparing suffixes SA[j - 1] and SA[j] directly over at most kLcpCap bytes
// (eight at a time); where they agree on all of them the entry is "long".
// Second, only for the long entries: with Phi[SA[j]] = SA[j - 1] (the suffix
// just before suffix i in sorted order), the permuted array PLCP[i] =
// lcp(suffix i, suffix Phi[i]) satisfies PLCP[i + 1] >= PLCP[i] - 1, so a
// left-to-right pass over the text positions extends each common prefix from
// the previous one minus one (Kasai et al.'s argument, in the Phi form of
// Kaerkkaeinen, Manzini and Puglisi), and a long one from at least kLcpCap.
// Each thread runs that pass over its own stretch of positions (skipping
// stretches without long positions, found in a bitmap); then LCP[j] =
// PLCP[SA[j]] for the long entries. Texts with short common prefixes take the
// first part almost alone; repetitive ones fall back to the second.
//
// FM index. Rows of the transform are the sorted suffixes of text$ (row 0 is
// $ alone, row r >= 1 is suffix SA[r - 1]); B[r] is the character before row
// r's suffix. C[c] = 1 + #{i : T[i] < c} is the first row starting with byte c
// and Occ(c, r) = #{q < r : B[q] = c}. Backward search keeps [sp, ep), the rows
// that start with the pattern's suffix read so far: sp = C[c] + Occ(c, sp),
// ep = C[c] + Occ(c, ep) for each pattern byte c from the last to the first.
// Occ comes from a table sampled every kOccBlock rows per byte present in the
// text plus a count over the rest of the block.

#include <cstring>
#include <vector>

#include "driver.h"

using namespace drv;

namespace {

constexpr u32 kNone = 0xFFFFFFFFu;  // no predecessor (SA[0]); never a position (n < 2^32)
constexpr int kLcpStretch = 512;     // positions per thread in the PLCP pass
constexpr u32 kLcpCap = 32;          // bytes compared in suffix array order
constexpr u32 kLcpLong = 0xFFFFFFFFu;  // LCP entry still to come from the PLCP pass
constexpr int kOccBlock = 256;       // rows per occurrence sample
constexpr int kOccGroup = 64;        // sample blocks per workgroup of the count kernel
constexpr int kScanChunk = 4096;     // entries per workgroup of the sample scan

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ inline void flag_error(u64* err) {
  atomicOr(reinterpret_cast<unsigned long long*>(err), (unsigned long long)kErrBounds);
}

// Length of the common prefix of text[x, n) and text[y, n), at most `cap`,
// comparing eight bytes at a time where whole aligned words around both
// stretches lie inside the text (byte by byte otherwise).
__device__ inline u32 common_prefix(const u8* __restrict__ text, u64 n, u64 x, u64 y, u32 cap) {
  u64 lim = n - (x > y ? x : y);
  if (lim > cap) lim = cap;
  const uintptr_t t0 = reinterpret_cast<uintptr_t>(text);
  const uintptr_t ax = (t0 + x) & ~uintptr_t(7), ay = (t0 + y) & ~uintptr_t(7);
  const u64 words = (lim + 7) / 8 + 1;  // aligned words covering lim bytes from either start
  if (ax >= t0 && ay >= t0 && ax + 8 * words <= t0 + n && ay + 8 * words <= t0 + n) {
    const u64* px = reinterpret_cast<const u64*>(ax);
    const u64* py = reinterpret_cast<const u64*>(ay);
    const u32 sx = u32(t0 + x - ax) * 8, sy = u32(t0 + y - ay) * 8;  // bit offsets
    u64 wx = px[0], wy = py[0];
    for (u64 k = 0; 8 * k < lim; ++k) {
      const u64 nx = px[k + 1], ny = py[k + 1];
      // Bytes [8k, 8k + 8) of each stretch, little-endian.
      const u64 vx = sx ? (wx >> sx) | (nx << (64 - sx)) : wx;
      const u64 vy = sy ? (wy >> sy) | (ny << (64 - sy)) : wy;
      const u64 d = vx ^ vy;
      if (d) {
        const u64 m = 8 * k + u64(__builtin_ctzll(d) / 8);
        return u32(m < lim ? m : lim);
      }
      wx = nx;
      wy = ny;
    }
    return u32(lim);
  }
  u32 m = 0;
  while (m < lim && text[x + m] == text[y + m]) ++m;
  return m;
}

// LCP in suffix array order up to kLcpCap; a long entry marks its position in
// `long_bits` and records Phi there.
__global__ __launch_bounds__(256) void lcp_direct_kernel(const u8* __restrict__ text, u64 n,
                                                         const u32* __restrict__ sa,
                                                         u32* __restrict__ lcp,
                                                         u32* __restrict__ phi,
                                                         u32* __restrict__ long_bits,
                                                         u64* __restrict__ err) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 j = u64(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += stride) {
    if (j == 0) {
      lcp[0] = 0;
      continue;
    }
    const u32 a = sa[j - 1], b = sa[j];
    if (a >= n || b >= n || a == b) {
      flag_error(err);
      lcp[j] = 0;
      continue;
    }
    const u32 m = common_prefix(text, n, a, b, kLcpCap);
    if (m < kLcpCap) {
      lcp[j] = m;
    } else {
      lcp[j] = kLcpLong;
      phi[b] = a;
      atomicOr(&long_bits[b >> 5], 1u << (b & 31u));
    }
  }
}

// PLCP at the long positions, over stretches of kLcpStretch positions, in
// place over Phi. A long position's common prefix is at least kLcpCap and at
// least the previous position's minus one when that one was long too.
__global__ __launch_bounds__(256) void plcp_long_kernel(const u8* __restrict__ text, u64 n,
                                                        const u32* __restrict__ long_bits,
                                                        u32* __restrict__ phi_plcp) {
  static_assert(kLcpStretch % 32 == 0, "whole bitmap words per stretch");
  const u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  const u64 lo = t * kLcpStretch;
  if (lo >= n) return;
  const u64 hi = lo + kLcpStretch < n ? lo + kLcpStretch : n;
  u64 l = 0;
  for (u64 w0 = lo; w0 < hi; w0 += 32) {
    u32 bits = long_bits[w0 >> 5];
    if (!bits) {
      l = 0;
      continue;
    }
    for (u64 i = w0; i < hi && i < w0 + 32; ++i) {
      if (!((bits >> (i - w0)) & 1u)) {
        l = 0;
        continue;
      }
      const u64 p = phi_plcp[i];
      if (l < kLcpCap) l = kLcpCap;
      // Extend eight bytes at a time while both stretches agree on all of them.
      for (;;) {
        const u64 room = n - (i > p ? i : p);
        if (l >= room) break;
        const u32 step = room - l < 4096 ? u32(room - l) : 4096u;
        const u32 m = common_prefix(text, n, i + l, p + l, step);
        l += m;
        if (m < step) break;
      }
      phi_plcp[i] = u32(l);
      l = l ? l - 1 : 0;
    }
  }
}

// LCP[j] = PLCP[SA[j]] for the long entries.
__global__ __launch_bounds__(256) void lcp_long_gather_kernel(const u32* __restrict__ sa, u64 n,
                                                              const u32* __restrict__ plcp,
                                                              u32* __restrict__ lcp) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 j = u64(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += stride) {
    if (lcp[j] != kLcpLong) continue;
    const u32 s = sa[j];
    lcp[j] = s < n ? plcp[s] : 0u;
  }
}

// The row of $ (1 + the j with SA[j] = 0) into *dollar.
__global__ __launch_bounds__(256) void find_dollar_kernel(const u32* __restrict__ sa, u64 n,
                                                          u64* __restrict__ dollar) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 j = u64(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += stride)
    if (sa[j] == 0) *dollar = j + 1;
}

// Transform rows r = 0 .. n: B[r] = T[n - 1] for r = 0, T[SA[r - 1] - 1]
// otherwise; the $ row either is left out (compact: rows after it move down by
// one) or holds the byte 0 (the FM index keeps every row and corrects its
// counts at the $ row).
__global__ __launch_bounds__(256) void bwt_kernel(const u8* __restrict__ text, u64 n,
                                                  const u32* __restrict__ sa,
                                                  const u64* __restrict__ dollar, int compact,
                                                  u8* __restrict__ out, u64* __restrict__ err) {
  const u64 d = *dollar;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 r = u64(blockIdx.x) * blockDim.x + threadIdx.x; r <= n; r += stride) {
    u8 ch = 0;
    if (r == 0) {
      ch = text[n - 1];
    } else {
      const u32 s = sa[r - 1];
      if (s >= n) {
        flag_error(err);
        continue;
      }
      if (s == 0) {
        if (!compact) out[r] = 0;
        continue;
      }
      ch = text[s - 1];
    }
    out[compact && r > d ? r - 1 : r] = ch;
  }
}

// Byte counts of the text (for C) in LDS, then one atomic per byte value.
__global__ __launch_bounds__(256) void byte_count_kernel(const u8* __restrict__ text, u64 n,
                                                         u64* __restrict__ counts) {
  __shared__ u32 h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    atomicAdd(&h[text[i]], 1u);
  __syncthreads();
  if (h[threadIdx.x])
    atomicAdd(reinterpret_cast<unsigned long long*>(counts + threadIdx.x),
              (unsigned long long)h[threadIdx.x]);
}

// Per sample block b (rows [b * kOccBlock, (b + 1) * kOccBlock) of B): the
// count of each present byte, written to occ[code][b] (a later scan turns the
// counts into prefix sums). A workgroup takes kOccGroup consecutive blocks so
// that each byte's row of counts is written in runs. The $ row (byte 0 in B)
// is not counted.
__global__ __launch_bounds__(256) void occ_count_kernel(const u8* __restrict__ B, u64 rows,
                                                        u64 nblocks, u64 dollar,
                                                        const u8* __restrict__ sym, u32 sigma,
                                                        u64 stride_b, u32* __restrict__ occ) {
  __shared__ u32 cnt[256][kOccGroup];
  for (int i = threadIdx.x; i < 256 * kOccGroup; i += 256) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const u64 b0 = u64(blockIdx.x) * kOccGroup;
  const u64 r0 = b0 * kOccBlock;
  constexpr int kBytes = kOccGroup * kOccBlock;  // rows of the group
  for (int q = threadIdx.x; q < kBytes; q += 256) {
    const u64 r = r0 + u64(q);
    if (r < rows && r != dollar) atomicAdd(&cnt[B[r]][q / kOccBlock], 1u);
  }
  __syncthreads();
  for (u32 idx = threadIdx.x; idx < sigma * kOccGroup; idx += 256) {
    const u32 c = idx / kOccGroup, g = idx % kOccGroup;
    const u64 b = b0 + g;
    if (b < nblocks) occ[u64(c) * stride_b + b] = cnt[sym[c]][g];
  }
}

// Exclusive scan of each byte's row of block counts, in three steps: chunks
// of kScanChunk entries scanned in LDS (chunk totals saved), the totals of a
// row scanned by one workgroup, the chunk offsets added.
__global__ __launch_bounds__(256) void occ_scan_chunks_kernel(u32* __restrict__ occ, u64 entries,
                                                              u64 stride_b, u64 chunks,
                                                              u64* __restrict__ totals) {
  __shared__ u32 wsum[4];
  const u64 c = blockIdx.y;
  const u64 ch = blockIdx.x;
  u32* row = occ + c * stride_b;
  const u64 base = ch * kScanChunk;
  constexpr int IT = kScanChunk / 256;
  u32 v[IT];
  u32 sum = 0;
  for (int k = 0; k < IT; ++k) {
    const u64 e = base + u64(threadIdx.x) * IT + k;
    v[k] = e < entries ? row[e] : 0u;
    sum += v[k];
  }
  // Exclusive scan of the per-thread sums.
  u32 inc = sum;
  for (int off = 1; off < kWave; off <<= 1) {
    const u32 t = __shfl_up(inc, off, kWave);
    if (lane_id() >= off) inc += t;
  }
  if (lane_id() == kWave - 1) wsum[threadIdx.x / kWave] = inc;
  __syncthreads();
  u32 woff = 0, total = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < int(threadIdx.x / kWave)) woff += wsum[w];
    total += wsum[w];
  }
  u32 run = woff + inc - sum;
  for (int k = 0; k < IT; ++k) {
    const u64 e = base + u64(threadIdx.x) * IT + k;
    if (e < entries) row[e] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) totals[c * chunks + ch] = total;
}

__global__ __launch_bounds__(64) void occ_scan_totals_kernel(u64* __restrict__ totals,
                                                             u64 chunks) {
  if (threadIdx.x != 0) return;
  u64* t = totals + u64(blockIdx.x) * chunks;
  u64 run = 0;
  for (u64 k = 0; k < chunks; ++k) {
    const u64 v = t[k];
    t[k] = run;
    run += v;
  }
}

__global__ __launch_bounds__(256) void occ_scan_add_kernel(u32* __restrict__ occ, u64 entries,
                                                           u64 stride_b, u64 chunks,
                                                           const u64* __restrict__ totals) {
  const u64 c = blockIdx.y;
  const u64 ch = blockIdx.x;
  const u32 add = u32(totals[c * chunks + ch]);
  u32* row = occ + c * stride_b;
  const u64 base = ch * kScanChunk;
  for (int k = threadIdx.x; k < kScanChunk; k += 256) {
    const u64 e = base + u64(k);
    if (e < entries) row[e] += add;
  }
}

// Occ(c, r) for one wave: the sample at r's block plus the matches of byte c
// among the block's rows before r (a wave reads the 256-row block as one
// 4-byte word per lane and counts with four ballots), minus the $ row when
// c is the byte 0 that stands in for it.
__device__ inline u64 occ_wave(const u8* __restrict__ B, const u32* __restrict__ occ_row,
                               u64 dollar, u32 c, u64 r) {
  const u64 b = r / kOccBlock;
  const u64 start = b * kOccBlock;
  const int lane = lane_id();
  const u32 word = reinterpret_cast<const u32*>(B + start)[lane];
  u64 part = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const u64 pos = start + u64(lane) * 4 + k;
    const bool hit = pos < r && ((word >> (8 * k)) & 0xFFu) == c;
    part += __popcll(__ballot(hit));
  }
  if (c == 0 && dollar >= start && dollar < r) part -= 1;
  return u64(occ_row[b]) + part;
}

// One wave per pattern; patterns concatenated with offsets[num + 1].
__global__ __launch_bounds__(256) void fm_count_kernel(
    const u8* __restrict__ B, u64 n, u64 dollar, const u32* __restrict__ occ, u64 stride_b,
    const u64* __restrict__ C, const u16* __restrict__ code, const u8* __restrict__ pats,
    const u64* __restrict__ offs, u32 num, u64* __restrict__ ranges) {
  const u64 waves = (u64(gridDim.x) * blockDim.x) / kWave;
  for (u64 q = (u64(blockIdx.x) * blockDim.x + threadIdx.x) / kWave; q < num; q += waves) {
    const u64 a = offs[q], z = offs[q + 1];
    u64 sp = 0, ep = n + 1;
    if (z > a) {
      for (u64 k = z; k-- > a;) {
        const u32 c = pats[k];
        const u32 cc = code[c];
        const u64 base = C[c];
        if (cc == 0xFFFFu) {
          sp = ep = base;  // the byte does not occur: no row starts with it
        } else {
          const u32* row = occ + u64(cc) * stride_b;
          sp = base + occ_wave(B, row, dollar, c, sp);
          ep = base + occ_wave(B, row, dollar, c, ep);
        }
      }
      // Rows 1.. are suffixes SA[0..]: the $ row never starts with a byte.
      sp -= 1;
      ep -= 1;
    } else {
      ep = n;  // the empty pattern: every suffix
    }
    if (lane_id() == 0) {
      ranges[2 * q] = sp;
      ranges[2 * q + 1] = ep;
    }
  }
}

u32 grid_for(u64 items, u32 per_block, u32 cap) {
  u64 g = ceil_div(std::max<u64>(items, 1), per_block);
  return u32(std::min<u64>(g, cap));
}

sa_status finish(sa_ctx* c, hipStream_t s) {
  // readback() also reports the kernels' error flag.
  return readback(c, s);
}

}  // namespace

// The FM index: the transform rows, the occurrence samples and the tables.
struct sa_fm {
  int device = 0;
  u64 n = 0, dollar = 0, nblocks = 0, stride_b = 0;
  u32 sigma = 0;
  void* dev = nullptr;
  u8* B = nullptr;
  u32* occ = nullptr;
  u64* C = nullptr;
  u16* code = nullptr;
};

extern "C" {

sa_status sa_lcp(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, const uint32_t* d_sa,
                 uint32_t* d_lcp, void* stream) {
  if (!ctx) return SA_EINVAL;
  if (n == 0) return SA_OK;
  if (!d_text || !d_sa || !d_lcp) return SA_EINVAL;
  if (n >= (u64(1) << 32)) return SA_ETOOBIG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipSetDevice(ctx->device) != hipSuccess) return SA_EDEVICE;
  sa_status st = ensure_workspace(ctx, n);
  if (st != SA_OK) return st;
  launch_fill_u64(ctx->counters, kCtrCount, 0, s);
  u32* phi = ctx->isa;        // Phi at the long positions, then PLCP in place
  u32* long_bits = ctx->live;  // the long positions
  launch_fill_u32(long_bits, ceil_div(n, 32), 0, s);
  const u32 g = grid_for(n, 256, 8192);
  hipLaunchKernelGGL(lcp_direct_kernel, dim3(g), dim3(256), 0, s, d_text, n, d_sa, d_lcp, phi,
                     long_bits, ctx->counters + kCtrError);
  const u64 threads = ceil_div(n, kLcpStretch);
  hipLaunchKernelGGL(plcp_long_kernel, dim3(u32(ceil_div(threads, 256))), dim3(256), 0, s,
                     d_text, n, long_bits, phi);
  hipLaunchKernelGGL(lcp_long_gather_kernel, dim3(g), dim3(256), 0, s, d_sa, n, phi, d_lcp);
  return finish(ctx, s);
}

sa_status sa_bwt(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, const uint32_t* d_sa,
                 uint8_t* d_bwt, uint64_t* dollar, void* stream) {
  if (!ctx || !dollar) return SA_EINVAL;
  *dollar = 0;
  if (n == 0) return SA_OK;
  if (!d_text || !d_sa || !d_bwt) return SA_EINVAL;
  if (n >= (u64(1) << 32)) return SA_ETOOBIG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipSetDevice(ctx->device) != hipSuccess) return SA_EDEVICE;
  launch_fill_u64(ctx->counters, kCtrCount, 0, s);
  u64* d_dollar = ctx->counters + kCtrIndexAux;
  const u32 g = grid_for(n + 1, 256, 8192);
  hipLaunchKernelGGL(find_dollar_kernel, dim3(g), dim3(256), 0, s, d_sa, n, d_dollar);
  hipLaunchKernelGGL(bwt_kernel, dim3(g), dim3(256), 0, s, d_text, n, d_sa, d_dollar, 1, d_bwt,
                     ctx->counters + kCtrError);
  const sa_status st = finish(ctx, s);
  if (st != SA_OK) return st;
  *dollar = ctx->h_counters[kCtrIndexAux];
  if (*dollar == 0 || *dollar > n) return SA_EDEVICE;  // SA holds no 0: not a suffix array
  return SA_OK;
}

sa_status sa_fm_create(sa_fm** out, sa_ctx* ctx, const uint8_t* d_text, uint64_t n,
                       const uint32_t* d_sa, void* stream) {
  if (!out || !ctx) return SA_EINVAL;
  *out = nullptr;
  if (n >= (u64(1) << 32)) return SA_ETOOBIG;
  if (n && (!d_text || !d_sa)) return SA_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipSetDevice(ctx->device) != hipSuccess) return SA_EDEVICE;
  sa_fm* fm = new (std::nothrow) sa_fm();
  if (!fm) return SA_ENOMEM;
  fm->device = ctx->device;
  fm->n = n;
  const u64 rows = n + 1;
  fm->nblocks = ceil_div(rows, kOccBlock) + 1;  // one more: Occ(c, rows) when rows % 256 == 0
  // Byte counts -> C, the present bytes and their codes (on the host: 256 values).
  std::vector<u64> counts(256, 0);
  u64* tmp = nullptr;
  if (!dev_alloc(&tmp, 256)) {
    delete fm;
    return SA_ENOMEM;
  }
  (void)hipMemsetAsync(tmp, 0, 256 * sizeof(u64), s);
  if (n)
    hipLaunchKernelGGL(byte_count_kernel, dim3(grid_for(n, 256 * 16, 2048)), dim3(256), 0, s,
                       d_text, n, tmp);
  if (hipMemcpyAsync(counts.data(), tmp, 256 * sizeof(u64), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(tmp);
    delete fm;
    return SA_EDEVICE;
  }
  std::vector<u64> C(256, 0);
  std::vector<u16> code(256, 0xFFFFu);
  std::vector<u8> sym;
  u64 run = 1;  // row 0 is $
  for (int c = 0; c < 256; ++c) {
    C[c] = run;
    run += counts[c];
    if (counts[c]) {
      code[c] = u16(sym.size());
      sym.push_back(u8(c));
    }
  }
  fm->sigma = u32(sym.size());
  fm->stride_b = (fm->nblocks + 63) / 64 * 64;
  const u64 chunks = ceil_div(fm->nblocks, kScanChunk);
  // One allocation: B (rows, padded to whole blocks), occ, C, code, sym, totals.
  const size_t b_bytes = (fm->nblocks * kOccBlock + 255) / 256 * 256;
  const size_t occ_bytes = size_t(std::max<u32>(fm->sigma, 1)) * fm->stride_b * 4;
  const size_t off_occ = b_bytes, off_C = off_occ + occ_bytes, off_code = off_C + 256 * 8,
               off_sym = off_code + 512, off_tot = off_sym + 256,
               total = off_tot + size_t(std::max<u32>(fm->sigma, 1)) * chunks * 8;
  if (hipMalloc(&fm->dev, total) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(tmp);
    delete fm;
    return SA_ENOMEM;
  }
  char* p = static_cast<char*>(fm->dev);
  fm->B = reinterpret_cast<u8*>(p);
  fm->occ = reinterpret_cast<u32*>(p + off_occ);
  fm->C = reinterpret_cast<u64*>(p + off_C);
  fm->code = reinterpret_cast<u16*>(p + off_code);
  u8* d_sym = reinterpret_cast<u8*>(p + off_sym);
  u64* totals = reinterpret_cast<u64*>(p + off_tot);
  sa_status st = SA_OK;
  if (hipMemsetAsync(fm->B, 0, b_bytes, s) != hipSuccess ||
      hipMemcpyAsync(fm->C, C.data(), 256 * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(fm->code, code.data(), 512, hipMemcpyHostToDevice, s) != hipSuccess ||
      (fm->sigma && hipMemcpyAsync(d_sym, sym.data(), fm->sigma, hipMemcpyHostToDevice, s) !=
                        hipSuccess))
    st = SA_EDEVICE;
  if (st == SA_OK && n) {
    launch_fill_u64(ctx->counters, kCtrCount, 0, s);
    u64* d_dollar = ctx->counters + kCtrIndexAux;
    const u32 g = grid_for(rows, 256, 8192);
    hipLaunchKernelGGL(find_dollar_kernel, dim3(g), dim3(256), 0, s, d_sa, n, d_dollar);
    hipLaunchKernelGGL(bwt_kernel, dim3(g), dim3(256), 0, s, d_text, n, d_sa, d_dollar, 0, fm->B,
                       ctx->counters + kCtrError);
    st = finish(ctx, s);
    if (st == SA_OK) {
      fm->dollar = ctx->h_counters[kCtrIndexAux];
      if (fm->dollar == 0 || fm->dollar > n) st = SA_EDEVICE;
    }
  }
  if (st == SA_OK && fm->sigma) {
    hipLaunchKernelGGL(occ_count_kernel, dim3(u32(ceil_div(fm->nblocks, kOccGroup))), dim3(256),
                       0, s, fm->B, rows, fm->nblocks, n ? fm->dollar : ~u64(0), d_sym,
                       fm->sigma, fm->stride_b, fm->occ);
    hipLaunchKernelGGL(occ_scan_chunks_kernel, dim3(u32(chunks), fm->sigma), dim3(256), 0, s,
                       fm->occ, fm->nblocks, fm->stride_b, chunks, totals);
    hipLaunchKernelGGL(occ_scan_totals_kernel, dim3(fm->sigma), dim3(64), 0, s, totals, chunks);
    hipLaunchKernelGGL(occ_scan_add_kernel, dim3(u32(chunks), fm->sigma), dim3(256), 0, s,
                       fm->occ, fm->nblocks, fm->stride_b, chunks, totals);
    if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) st = SA_EDEVICE;
  }
  (void)hipFree(tmp);
  if (st != SA_OK) {
    sa_fm_destroy(fm);
    return st;
  }
  *out = fm;
  return SA_OK;
}

sa_status sa_fm_count(sa_fm* fm, const uint8_t* d_patterns, const uint64_t* d_offsets,
                      uint32_t num_patterns, uint64_t* d_ranges, void* stream) {
  if (!fm) return SA_EINVAL;
  if (num_patterns == 0) return SA_OK;
  if (!d_offsets || !d_ranges) return SA_EINVAL;
  if (hipSetDevice(fm->device) != hipSuccess) return SA_EDEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const u64 waves_per_block = 256 / kWave;
  const u32 g = grid_for(num_patterns, u32(waves_per_block), 16384);
  hipLaunchKernelGGL(fm_count_kernel, dim3(g), dim3(256), 0, s, fm->B, fm->n, fm->dollar,
                     fm->occ, fm->stride_b, fm->C, fm->code, d_patterns, d_offsets, num_patterns,
                     d_ranges);
  if (hipGetLastError() != hipSuccess) return SA_EDEVICE;
  return SA_OK;
}

sa_status sa_fm_info(const sa_fm* fm, uint64_t* n, uint64_t* dollar, uint32_t* sigma,
                     uint64_t* device_bytes) {
  if (!fm) return SA_EINVAL;
  if (n) *n = fm->n;
  if (dollar) *dollar = fm->dollar;
  if (sigma) *sigma = fm->sigma;
  if (device_bytes) {
    const u64 chunks = ceil_div(fm->nblocks, kScanChunk);
    *device_bytes = (fm->nblocks * kOccBlock + 255) / 256 * 256 +
                    u64(std::max<u32>(fm->sigma, 1)) * fm->stride_b * 4 + 256 * 8 + 512 + 256 +
                    u64(std::max<u32>(fm->sigma, 1)) * chunks * 8;
  }
  return SA_OK;
}

sa_status sa_fm_destroy(sa_fm* fm) {
  if (!fm) return SA_OK;
  (void)hipSetDevice(fm->device);
  (void)hipFree(fm->dev);
  delete fm;
  return SA_OK;
}

}  // extern "C"
