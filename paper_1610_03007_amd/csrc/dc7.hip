// Suffix array by the difference cover algorithm DC7 (Section 2.2): the sample
// is the suffixes at positions i mod 7 in D7 = {0, 1, 3}, three in every seven,
// so its string of names is 3/7 of the text. For any two positions i, j there
// is an offset k < 7 with (i + k) mod 7 and (j + k) mod 7 both in D7, so any two
// suffixes compare by at most k characters and then two sample ranks.
//
//   1. The sample as the string x0 x1 x3 (positions 0, 7, 14, ... then 1, 8,
//      ... then 3, 10, ...), each entry named by its seven characters
//      (9 bits each with the sentinel below every byte: 63-bit radix keys).
//      A part whose last tuple has no sentinel (n mod 7 == 0 for x0, 1 for x1)
//      ends with a dummy position n: an all-sentinel tuple, unique and the
//      smallest, so that no suffix of the name string compares across parts.
//   2. The sample's suffix order: from the sorted tuples when the names are
//      unique, else by DC3 on the name string.
//   3. The four other classes (2, 4, 5, 6 mod 7) in one radix sort, keyed by
//      (class, the characters up to the next sample position, its rank).
//   4. Five sorted lists (four classes and the sample by rank) merged pairwise
//      along the merge path, with the comparison above on 24-byte records of
//      seven characters and the ranks of the three sample positions they span.

#include "driver.h"

namespace sa {

constexpr u32 kD7 = (1u << 0) | (1u << 1) | (1u << 3);

__host__ __device__ inline bool d7_in(u32 c) { return (kD7 >> c) & 1u; }
// Rank slot of a cover class: 0 -> 0, 1 -> 1, 3 -> 2.
__host__ __device__ inline u32 d7_slot(u32 c) { return c == 0 ? 0u : c == 1 ? 1u : 2u; }
// Smallest k < 7 with (a + k) mod 7 and (b + k) mod 7 both in D7.
__host__ __device__ inline u32 d7_offset(u32 a, u32 b) {
  for (u32 k = 0; k < 7; ++k)
    if (d7_in((a + k) % 7) && d7_in((b + k) % 7)) return k;
  return 7;  // not reached: D7 is a difference cover modulo 7
}

struct D7Text {
  const u8* t;
  u64 n;
  __device__ u64 sym(u64 p) const { return p < n ? u64(t[p]) + 1 : 0; }
  // Characters p .. p + k - 1, 9 bits each, the first most significant.
  __device__ u64 chars(u64 p, u32 k) const {
    u64 v = 0;
    for (u32 q = 0; q < k; ++q) v = (v << 9) | sym(p + q);
    return v;
  }
};

struct D7Layout {
  u64 n0, n1, n3;  // entries of x0, x1, x3 (dummies included)
  u32 dummy;       // 1 if x0 or x1 ends with the dummy position n
  __host__ __device__ u64 pos(u64 s) const {
    if (s < n0) return 7 * s;
    if (s < n0 + n1) return 7 * (s - n0) + 1;
    return 7 * (s - n0 - n1) + 3;
  }
};

__global__ __launch_bounds__(256) void d7_pack_sample_kernel(D7Text txt, D7Layout L, u64 ms,
                                                            u64* __restrict__ keys,
                                                            u32* __restrict__ vals) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 s = u64(blockIdx.x) * blockDim.x + threadIdx.x; s < ms; s += stride) {
    keys[s] = txt.chars(L.pos(s), 7);
    vals[s] = u32(s);
  }
}

__global__ __launch_bounds__(256) void d7_ranks_kernel(const u32* __restrict__ sa_s, u64 ms,
                                                      D7Layout L, u64 n, u32* __restrict__ rankp,
                                                      u32* __restrict__ byrank,
                                                      u64* __restrict__ counters) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  bool bad = false;
  for (u64 j = u64(blockIdx.x) * blockDim.x + threadIdx.x; j < ms; j += stride) {
    const u64 s = sa_s[j];
    const u64 p = s < ms ? L.pos(s) : ~u64(0);
    if (j < L.dummy) {
      bad |= p != n;  // the dummy's all-sentinel tuple is the smallest
      continue;
    }
    if (p >= n) {
      bad = true;
      continue;
    }
    rankp[p] = u32(j + 1 - L.dummy);
    byrank[j - L.dummy] = u32(p);
  }
  if (bad)
    atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
             (unsigned long long)kErrBounds);
}

__device__ inline u64 d7_rank(const u32* __restrict__ rankp, u64 n, u64 p) {
  return p < n ? rankp[p] : 0;
}

// Non-sample position t of nns: the full blocks of seven hold classes 2, 4, 5
// and 6 in order, the last block those below n.
__device__ inline u64 d7_nonsample_pos(u64 t) {
  const u32 cls[4] = {2, 4, 5, 6};
  return 7 * (t >> 2) + cls[t & 3];
}

// Offset of the next sample position from classes 2, 4, 5, 6: 1, 3, 2, 1.
__global__ __launch_bounds__(256) void d7_pack_rest_kernel(D7Text txt, u64 nns,
                                                          const u32* __restrict__ rankp,
                                                          u64* __restrict__ keys,
                                                          u32* __restrict__ vals) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x; t < nns; t += stride) {
    const u64 p = d7_nonsample_pos(t);
    const u32 ci = u32(t & 3);
    const u32 k = ci == 1 ? 3u : ci == 2 ? 2u : 1u;
    keys[t] = (u64(ci) << 60) | (txt.chars(p, k) << 32) | d7_rank(rankp, txt.n, p + k);
    vals[t] = u32(p);
  }
}

struct D7Rec {
  u64 chars;   // characters p .. p + 6
  u32 rk[3];   // ranks of the sample positions in p .. p + 6, by cover class
  u32 pos;
};

__device__ inline D7Rec d7_rec(const D7Text& txt, const u32* __restrict__ rankp, u64 p) {
  D7Rec r;
  r.chars = txt.chars(p, 7);
  const u32 a = u32(p % 7);
  r.rk[0] = u32(d7_rank(rankp, txt.n, p + (7 - a) % 7));
  r.rk[1] = u32(d7_rank(rankp, txt.n, p + (8 - a) % 7));
  r.rk[2] = u32(d7_rank(rankp, txt.n, p + (10 - a) % 7));
  r.pos = u32(p);
  return r;
}

__device__ inline bool d7_less(const D7Rec& x, const D7Rec& y) {
  const u32 a = x.pos % 7, b = y.pos % 7;
  const u32 k = d7_offset(a, b);
  if (k > 0) {
    const u64 cx = x.chars >> (9 * (7 - k)), cy = y.chars >> (9 * (7 - k));
    if (cx != cy) return cx < cy;
  }
  return x.rk[d7_slot((a + k) % 7)] < y.rk[d7_slot((b + k) % 7)];
}

// Records of the sorted non-sample suffixes (the sort's final value buffer)
// followed by those of the sample in rank order.
__global__ __launch_bounds__(256) void d7_records_kernel(
    D7Text txt, u64 nns, u64 nsr, const u32* __restrict__ vA, const u32* __restrict__ vB,
    const SortPlan* __restrict__ plan, const u32* __restrict__ rankp,
    const u32* __restrict__ byrank, D7Rec* __restrict__ rec) {
  const u32* rest = plan->final_buf ? vB : vA;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x; t < nns + nsr; t += stride)
    rec[t] = d7_rec(txt, rankp, t < nns ? rest[t] : byrank[t - nns]);
}

constexpr int kD7Items = 4;
constexpr int kD7Tile = 256 * kD7Items;

// Merge path of two sorted record lists a[0, na) and b[0, nb).
__global__ __launch_bounds__(256) void d7_partition_kernel(const D7Rec* __restrict__ a, u64 na,
                                                          const D7Rec* __restrict__ b, u64 nb,
                                                          u64 ntiles, u64* __restrict__ split) {
  const u64 m = na + nb;
  for (u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x; t <= ntiles;
       t += u64(gridDim.x) * blockDim.x) {
    const u64 d = t * kD7Tile < m ? t * kD7Tile : m;
    u64 lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
      const u64 mid = (lo + hi) >> 1;
      if (d7_less(a[mid], b[d - 1 - mid]))
        lo = mid + 1;
      else
        hi = mid;
    }
    split[t] = lo;
  }
}

// One workgroup per tile of the merged output: both input runs in LDS, each
// thread merges kD7Items records from its start on the merge path. Writes the
// merged records, or (out_pos set) only their positions.
__global__ __launch_bounds__(256) void d7_merge_tile_kernel(
    const D7Rec* __restrict__ a, u64 na, const D7Rec* __restrict__ b, u64 nb,
    const u64* __restrict__ split, D7Rec* __restrict__ out, u32* __restrict__ out_pos,
    u64* __restrict__ counters) {
  __shared__ D7Rec s_a[kD7Tile], s_b[kD7Tile];
  const u64 m = na + nb;
  const u64 t = blockIdx.x;
  const u64 d0 = t * kD7Tile;
  const u64 d1 = d0 + kD7Tile < m ? d0 + kD7Tile : m;
  const u64 a0 = split[t], a1 = split[t + 1];
  const u64 b0 = d0 - a0, b1 = d1 - a1;
  const u32 ka = u32(a1 - a0), kb = u32(b1 - b0), nt = u32(d1 - d0);
  if (a1 < a0 || b1 < b0 || a1 > na || b1 > nb || ka + kb != nt || nt > u32(kD7Tile)) {
    if (threadIdx.x == 0)
      atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
               (unsigned long long)kErrBounds);
    return;
  }
  for (u32 k = threadIdx.x; k < ka; k += blockDim.x) s_a[k] = a[a0 + k];
  for (u32 k = threadIdx.x; k < kb; k += blockDim.x) s_b[k] = b[b0 + k];
  __syncthreads();
  const u32 dd = threadIdx.x * kD7Items;
  if (dd >= nt) return;
  u32 lo = dd > kb ? dd - kb : 0, hi = dd < ka ? dd : ka;
  while (lo < hi) {
    const u32 mid = (lo + hi) >> 1;
    if (d7_less(s_a[mid], s_b[dd - 1 - mid]))
      lo = mid + 1;
    else
      hi = mid;
  }
  u32 ia = lo, ib = dd - lo;
#pragma unroll
  for (int k = 0; k < kD7Items; ++k) {
    if (dd + k >= nt) break;
    const bool take_a = ib >= kb || (ia < ka && d7_less(s_a[ia], s_b[ib]));
    const D7Rec& r = take_a ? s_a[ia++] : s_b[ib++];
    if (out_pos)
      out_pos[d0 + dd + k] = r.pos;
    else
      out[d0 + dd + k] = r;
  }
}

}  // namespace sa

namespace drv {

struct D7Arrays {
  u32* child = nullptr;
  u32* childsa = nullptr;
  u32* tmp = nullptr;
  u32* rankp = nullptr;
  u32* byrank = nullptr;
  D7Rec* rec = nullptr;
  D7Rec* rec2 = nullptr;
  u64* split = nullptr;
};

// Merges a[0, na) and b[0, nb) into out (records) or out_pos (positions).
void d7_merge(sa_ctx* c, const D7Rec* a, u64 na, const D7Rec* b, u64 nb, D7Rec* out,
              u32* out_pos, u64* split, hipStream_t s) {
  const u64 m = na + nb;
  if (m == 0) return;
  const u64 ntiles = ceil_div(m, u64(kD7Tile));
  Tracer t(c, s, SA_KERNEL_OTHER, double(m) * (out_pos ? 28.0 : 48.0));
  hipLaunchKernelGGL(d7_partition_kernel, dim3(u32(ceil_div(ntiles + 1, 256))), dim3(256), 0, s,
                     a, na, b, nb, ntiles, split);
  hipLaunchKernelGGL(d7_merge_tile_kernel, dim3(u32(ntiles)), dim3(256), 0, s, a, na, b, nb, split,
                     out, out_pos, c->counters);
}

sa_status build_dc7(sa_ctx* c, const u8* text, u64 n, u32* d_sa, u32* d_rank, hipStream_t s) {
  std::memset(&c->info, 0, sizeof(c->info));
  c->info.n = n;
  if (n == 0) return SA_OK;
  if (!text || !d_sa) return SA_EINVAL;
  if (n >= (u64(1) << 32)) return SA_ETOOBIG;
  if (hipSetDevice(c->device) != hipSuccess) return SA_EDEVICE;
  resolve_tuning(c, "single", n, 0);
  sa_status st = ensure_workspace(c, n);
  if (st != SA_OK) return st;
  launch_fill_u64(c->counters, kCtrCount, 0, s);
  sa_build_info& info = c->info;
  info.rounds = 1;
  info.active[0] = n;

  const D7Text txt{text, n};
  auto count_of = [n](u64 cls) { return n > cls ? (n - cls + 6) / 7 : u64(0); };
  D7Layout L;
  const u32 d0 = n % 7 == 0 ? 1u : 0u, d1 = n % 7 == 1 ? 1u : 0u;
  L.n0 = count_of(0) + d0;
  L.n1 = count_of(1) + d1;
  L.n3 = count_of(3);
  L.dummy = d0 + d1;
  const u64 ms = L.n0 + L.n1 + L.n3;
  const u64 nsr = ms - L.dummy;  // real sample suffixes
  const u64 nns = n - nsr;       // the other classes
  D7Arrays A;
  // Depth 0, slots 10..17 (DC3's own levels use slots 0..8 and, under DC7,
  // depths from 1).
  if (!level_alloc(c, 0, 10, ms, &A.child) || !level_alloc(c, 0, 11, ms, &A.tmp) ||
      !level_alloc(c, 0, 12, n + 8, &A.rankp) || !level_alloc(c, 0, 13, nsr, &A.byrank) ||
      !level_alloc(c, 0, 14, n, &A.rec) || !level_alloc(c, 0, 15, n, &A.rec2) ||
      !level_alloc(c, 0, 16, ceil_div(n, u64(kD7Tile)) + 1, &A.split))
    return SA_ENOMEM;
  launch_fill_u32(A.rankp, n + 8, 0, s);
  const Bufs full = full_bufs(c);

  // Steps 1-2: name the sample's seven-character tuples; order the sample.
  {
    Tracer t(c, s, SA_KERNEL_PACK_TEXT, double(ms) * 19.0);
    hipLaunchKernelGGL(d7_pack_sample_kernel, dim3(stream_grid(c, ms, 256)), dim3(256), 0, s, txt,
                       L, ms, full.kA, full.vA);
  }
  run_sort(c, full, ms, npass_for(c, 63), 1, 0, s);
  {
    // The re-rank's first-round form: names into `child`, the order of unique
    // ones into tmp, the others counted.
    Tracer t(c, s, SA_KERNEL_RERANK, double(ms) * 16.0);
    const RerankArgs a = single_args(ms, ms, 0, kRerankScatterIsa);
    const u32 grid = u32(std::min<u64>(std::max<u64>(1, ceil_div(ms, kRerankTile)),
                                       u64(c->num_cus) * rerank_wgs_per_cu(false)));
    launch_rerank_compact(full.kA, full.kB, full.vA, full.vB, c->plan, a, c->ctl, A.child, A.tmp,
                          c->act_idx, nullptr, c->act_rank, c->counters, grid, s);
  }
  st = readback(c, s);
  if (st != SA_OK) return st;
  const u32* sa_s = A.tmp;
  if (c->h_counters[kCtrActive] > 0) {
    if (!level_alloc(c, 0, 17, ms, &A.childsa)) return SA_ENOMEM;
    st = dc3_names(c, A.child, ms, ms, A.childsa, 1, s);
    if (st != SA_OK) return st;
    sa_s = A.childsa;
  }
  hipLaunchKernelGGL(d7_ranks_kernel, dim3(scatter_grid(c, ms)), dim3(256), 0, s, sa_s, ms, L,
                     n, A.rankp, A.byrank, c->counters);

  // Step 3: the other four classes, by (class, characters to the next sample
  // position, its rank).
  if (nns > 0) {
    {
      Tracer t(c, s, SA_KERNEL_PACK_TEXT, double(nns) * 19.0);
      hipLaunchKernelGGL(d7_pack_rest_kernel, dim3(stream_grid(c, nns, 256)), dim3(256), 0, s,
                         txt, nns, A.rankp, full.kA, full.vA);
    }
    run_sort(c, full, nns, npass_for(c, 62), 1, 0, s);
  }

  // Step 4: records, then the merges (2 with 4, 5 with 6, those two, and the
  // result with the sample).
  {
    Tracer t(c, s, SA_KERNEL_OTHER, double(n) * 36.0);
    hipLaunchKernelGGL(d7_records_kernel, dim3(stream_grid(c, n, 256)), dim3(256), 0, s, txt, nns,
                       nsr, full.vA, full.vB, c->plan, A.rankp, A.byrank, A.rec);
  }
  const u64 c2 = count_of(2), c4 = count_of(4), c5 = count_of(5), c6 = count_of(6);
  const D7Rec* r2 = A.rec;
  const D7Rec* r4 = r2 + c2;
  const D7Rec* r5 = r4 + c4;
  const D7Rec* r6 = r5 + c5;
  const D7Rec* rs = A.rec + nns;
  d7_merge(c, r2, c2, r4, c4, A.rec2, nullptr, A.split, s);
  d7_merge(c, r5, c5, r6, c6, A.rec2 + c2 + c4, nullptr, A.split, s);
  d7_merge(c, A.rec2, c2 + c4, A.rec2 + c2 + c4, c5 + c6, A.rec, nullptr, A.split, s);
  d7_merge(c, A.rec, nns, rs, nsr, nullptr, d_sa, A.split, s);
  if (d_rank)
    if (hipMemcpyAsync(d_rank, A.rankp, n * sizeof(u32), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return SA_EDEVICE;
  // Waits for the build and checks the error flags.
  return readback(c, s);
}

}  // namespace drv

using namespace drv;

extern "C" {

sa_status sa_build_dc7(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t* d_sa,
                       uint32_t* d_rank_sample, void* stream) {
  if (!ctx) return SA_EINVAL;
  const sa_status st =
      build_dc7(ctx, d_text, n, d_sa, d_rank_sample, static_cast<hipStream_t>(stream));
  settle_trace(ctx, st);
  return st;
}

}  // extern "C"
