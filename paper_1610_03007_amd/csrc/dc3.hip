// Suffix array by the difference cover algorithm DC3 (Section 2.2, Alg. 7;
// Kaerkkaeinen, Sanders and Burkhardt): a second suffix sorter besides prefix
// doubling. One level on a string x of length m (symbols >= 1, 0 past the end):
//
//   1. The sample: positions i with i mod 3 != 0, as the string
//      x1 = [1, 4, 7, ...] followed by x2 = [2, 5, 8, ...]; x1 has ceil(m / 3)
//      entries, so when m mod 3 == 1 its last one is the position m itself (a
//      dummy whose triple is all sentinels: the smallest, and unique).
//   2. Sort the sample by its character triples (x[i], x[i+1], x[i+2]) and
//      name every triple by its head rank. If the names are unique, the sorted
//      order is the sample's suffix order; otherwise the names, in string order
//      x1 x2, are the string of the next level, whose suffix array gives it.
//   3. The ranks of the sample suffixes by position; the suffixes at i mod 3
//      == 0 sorted by (x[i], rank of i + 1).
//   4. Merge the two sorted lists with the comparison of the method: against a
//      suffix j = 1 mod 3, compare (x[i], rank(i+1)); against j = 2 mod 3,
//      (x[i], x[i+1], rank(i+2)) -- each side reaches a sample rank, so no
//      comparison ties. The merge splits the output into tiles along the merge
//      path (a binary search per tile boundary) and merges each tile in LDS.
//
// The sorts are the library's LSD radix sort. A triple of b-bit symbols fits a
// 64-bit key while 3b <= 64 (the bytes of the text: 27 bits); wider levels
// sort it as two words, (x[i+1], x[i+2]) first and then x[i] with the first
// word's run names as tie words, exactly as the quadrupling rounds do.

#include "driver.h"

namespace sa {

template <typename T>
struct Dc3Str {
  const T* x;
  u64 m;
  u32 add;  // 1 for the text's bytes (so that symbols are >= 1), 0 for names
  __device__ u64 sym(u64 p) const { return p < m ? u64(x[p]) + add : 0; }
};

// Position of sample index s: x1 (s < n0) then x2.
__host__ __device__ inline u64 dc3_pos(u64 s, u64 n0) {
  return s < n0 ? 3 * s + 1 : 3 * (s - n0) + 2;
}

// Triple keys of the sample (WORDS == 1: the whole triple; WORDS == 2: the
// low word (x[p+1], x[p+2])); values = sample index.
template <typename T, int WORDS>
__global__ __launch_bounds__(256) void dc3_pack_kernel(Dc3Str<T> str, u64 m12, u64 n0, int bsym,
                                                       u64* __restrict__ keys,
                                                       u32* __restrict__ vals) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 s = u64(blockIdx.x) * blockDim.x + threadIdx.x; s < m12; s += stride) {
    const u64 p = dc3_pos(s, n0);
    const u64 lo = (str.sym(p + 1) << bsym) | str.sym(p + 2);
    keys[s] = WORDS == 1 ? ((str.sym(p) << (2 * bsym)) | lo) : lo;
    vals[s] = u32(s);
  }
}

// High word of a two-word triple sort: x[p] for the sample index in pk.
template <typename T>
__global__ __launch_bounds__(256) void dc3_pack_hi_kernel(Dc3Str<T> str,
                                                          const SortCtl* __restrict__ ctl,
                                                          u64 n0, const u64* __restrict__ pk,
                                                          u64* __restrict__ keys) {
  const u64 count = ctl->count;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 q = u64(blockIdx.x) * blockDim.x + threadIdx.x; q < count; q += stride)
    keys[q] = str.sym(dc3_pos(u64(u32(pk[q])), n0));
}

// Sample ranks by position from the sample's suffix order sa12 (sample
// indices): rankp[p] = 1-based rank among the real sample suffixes (the dummy,
// when present, is first and is skipped) and byrank[r - 1] = p.
__global__ __launch_bounds__(256) void dc3_ranks_kernel(const u32* __restrict__ sa12, u64 m12,
                                                        u64 n0, u64 m, u32 dummy,
                                                        u32* __restrict__ rankp,
                                                        u32* __restrict__ byrank,
                                                        u64* __restrict__ counters) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  bool bad = false;
  for (u64 j = u64(blockIdx.x) * blockDim.x + threadIdx.x; j < m12; j += stride) {
    const u64 s = sa12[j];
    const u64 p = s < m12 ? dc3_pos(s, n0) : ~u64(0);
    if (j < dummy) {
      bad |= p != m;  // the dummy's all-sentinel triple is the smallest
      continue;
    }
    if (p >= m) {
      bad = true;
      continue;
    }
    rankp[p] = u32(j + 1 - dummy);
    byrank[j - dummy] = u32(p);
  }
  if (bad)
    atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
             (unsigned long long)kErrBounds);
}

// The suffixes at i mod 3 == 0, keyed (x[i], rank of i + 1).
template <typename T>
__global__ __launch_bounds__(256) void dc3_pack_s0_kernel(Dc3Str<T> str, u64 n0,
                                                          const u32* __restrict__ rankp,
                                                          int brank, u64* __restrict__ keys,
                                                          u32* __restrict__ vals) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 a = u64(blockIdx.x) * blockDim.x + threadIdx.x; a < n0; a += stride) {
    const u64 i = 3 * a;
    const u64 r1 = i + 1 < str.m ? rankp[i + 1] : 0;
    keys[a] = (str.sym(i) << brank) | r1;
    vals[a] = u32(i);
  }
}

template <typename T>
__device__ inline u64 dc3_rank(const Dc3Str<T>& str, const u32* __restrict__ rankp, u64 p) {
  return p < str.m ? rankp[p] : 0;
}

// Step 4, merge. Every suffix of both sorted lists gets a comparison record
// (x[p], x[p+1], rank(p+1), rank(p+2)) and its position; a mod-0 record A
// and a sample record B compare as the method says: against B at j = 1 mod 3,
// (x, rank(p+1)); against j = 2 mod 3, (x, x[p+1], rank(p+2)). Records are
// gathered once (random reads), then the merge reads them in order.
struct Dc3Rec {
  u32 c0, c1, r1, r2;
};

template <typename T>
__device__ inline Dc3Rec dc3_rec(const Dc3Str<T>& str, const u32* __restrict__ rankp, u64 p) {
  return Dc3Rec{u32(str.sym(p)), u32(str.sym(p + 1)), u32(dc3_rank(str, rankp, p + 1)),
                u32(dc3_rank(str, rankp, p + 2))};
}

// A (mod 0) below B (sample suffix at position pb).
__device__ inline bool dc3_rec_less(const Dc3Rec& a, const Dc3Rec& b, u64 pb) {
  if (a.c0 != b.c0) return a.c0 < b.c0;
  if (pb % 3 == 1) return a.r1 < b.r1;
  if (a.c1 != b.c1) return a.c1 < b.c1;
  return a.r2 < b.r2;
}

template <typename T>
__global__ __launch_bounds__(256) void dc3_records_kernel(
    Dc3Str<T> str, u64 n0, u64 n12, const u32* __restrict__ vA, const u32* __restrict__ vB,
    const SortPlan* __restrict__ plan, const u32* __restrict__ rankp,
    const u32* __restrict__ byrank, Dc3Rec* __restrict__ rec0, u32* __restrict__ pos0,
    Dc3Rec* __restrict__ rec12) {
  const u32* s0 = plan->final_buf ? vB : vA;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x; t < n0 + n12; t += stride) {
    if (t < n0) {
      const u32 i = s0[t];
      pos0[t] = i;
      rec0[t] = dc3_rec(str, rankp, i);
    } else {
      rec12[t - n0] = dc3_rec(str, rankp, byrank[t - n0]);
    }
  }
}

// Merge path: split[t] = how many mod-0 suffixes are among the first
// min(t * tile, m) suffixes of the merged order.
__global__ __launch_bounds__(256) void dc3_partition_kernel(
    const Dc3Rec* __restrict__ rec0, const Dc3Rec* __restrict__ rec12,
    const u32* __restrict__ byrank, u64 n0, u64 n12, u64 tile, u64 ntiles,
    u64* __restrict__ split) {
  const u64 m = n0 + n12;
  for (u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x; t <= ntiles;
       t += u64(gridDim.x) * blockDim.x) {
    const u64 d = t * tile < m ? t * tile : m;
    u64 lo = d > n12 ? d - n12 : 0, hi = d < n0 ? d : n0;
    while (lo < hi) {
      const u64 mid = (lo + hi) >> 1;
      const u64 b = d - 1 - mid;
      if (dc3_rec_less(rec0[mid], rec12[b], byrank[b]))
        lo = mid + 1;
      else
        hi = mid;
    }
    split[t] = lo;
  }
}

// One workgroup per tile of kDc3Tile merged suffixes: both input runs in LDS,
// each thread finds its start on the merge path and merges kDc3Items
// suffixes, and the tile's part of the suffix array is written in order.
constexpr int kDc3Items = 4;
constexpr int kDc3Tile = 256 * kDc3Items;

__global__ __launch_bounds__(256) void dc3_merge_tile_kernel(
    const Dc3Rec* __restrict__ rec0, const u32* __restrict__ pos0,
    const Dc3Rec* __restrict__ rec12, const u32* __restrict__ byrank,
    const u64* __restrict__ split, u64 n0, u64 n12, u32* __restrict__ sa,
    u64* __restrict__ counters) {
  __shared__ Dc3Rec s_a[kDc3Tile], s_b[kDc3Tile];
  __shared__ u32 s_pa[kDc3Tile], s_pb[kDc3Tile], s_out[kDc3Tile];
  const u64 m = n0 + n12;
  const u64 t = blockIdx.x;
  const u64 d0 = t * kDc3Tile;
  const u64 d1 = d0 + kDc3Tile < m ? d0 + kDc3Tile : m;
  const u64 a0 = split[t], a1 = split[t + 1];
  const u64 b0 = d0 - a0, b1 = d1 - a1;
  const u32 na = u32(a1 - a0), nb = u32(b1 - b0), nt = u32(d1 - d0);
  if (a1 < a0 || b1 < b0 || na + nb != nt || nt > u32(kDc3Tile)) {
    if (threadIdx.x == 0)
      atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
               (unsigned long long)kErrBounds);
    return;
  }
  for (u32 k = threadIdx.x; k < na; k += blockDim.x) {
    s_a[k] = rec0[a0 + k];
    s_pa[k] = pos0[a0 + k];
  }
  for (u32 k = threadIdx.x; k < nb; k += blockDim.x) {
    s_b[k] = rec12[b0 + k];
    s_pb[k] = byrank[b0 + k];
  }
  __syncthreads();
  const u32 dd = threadIdx.x * kDc3Items;
  if (dd < nt) {
    u32 lo = dd > nb ? dd - nb : 0, hi = dd < na ? dd : na;
    while (lo < hi) {
      const u32 mid = (lo + hi) >> 1;
      const u32 b = dd - 1 - mid;
      if (dc3_rec_less(s_a[mid], s_b[b], s_pb[b]))
        lo = mid + 1;
      else
        hi = mid;
    }
    u32 ia = lo, ib = dd - lo;
#pragma unroll
    for (int k = 0; k < kDc3Items; ++k) {
      if (dd + k >= nt) break;
      const bool take_a = ib >= nb || (ia < na && dc3_rec_less(s_a[ia], s_b[ib], s_pb[ib]));
      s_out[dd + k] = take_a ? s_pa[ia++] : s_pb[ib++];
    }
  }
  __syncthreads();
  for (u32 k = threadIdx.x; k < nt; k += blockDim.x) sa[d0 + k] = s_out[k];
}

// rank12[p] = rankp[p] for sample positions, 0 at positions divisible by 3.
__global__ __launch_bounds__(256) void dc3_rank_out_kernel(const u32* __restrict__ rankp, u64 m,
                                                           u32* __restrict__ out) {
  const u64 stride = u64(gridDim.x) * blockDim.x;
  for (u64 p = u64(blockIdx.x) * blockDim.x + threadIdx.x; p < m; p += stride)
    out[p] = p % 3 ? rankp[p] : 0u;
}

}  // namespace sa

namespace drv {

struct Dc3Level {
  u32* child = nullptr;   // the next level's string (names in x1 x2 order)
  u32* childsa = nullptr; // its suffix array
  u32* tmp = nullptr;     // sorted order when the names are unique
  u32* rankp = nullptr;   // sample ranks by position
  u32* byrank = nullptr;  // sample positions by rank
  Dc3Rec* rec0 = nullptr;  // comparison records of the sorted mod-0 suffixes
  Dc3Rec* rec12 = nullptr; // and of the sample suffixes by rank
  u32* pos0 = nullptr;
  u64* split = nullptr;    // merge-path splits
};

template <typename T>
sa_status dc3_level(sa_ctx* c, const T* x, u64 m, u32 add, u64 max_sym, u32* sa, u32* rank_out,
                    u32 depth, hipStream_t s) {
  if (m == 0) return SA_OK;
  if (depth >= u32(SA_MAX_ROUNDS)) return SA_EDEVICE;
  sa_build_info& info = c->info;
  info.rounds = std::max(info.rounds, depth + 1);
  info.active[depth] = m;
  if (m == 1) {
    launch_set_zero_u32(sa, s);
    if (rank_out) launch_fill_u32(rank_out, 1, 0, s);
    return SA_OK;
  }
  const Dc3Str<T> str{x, m, add};
  const u64 n0 = ceil_div(m, 3), n1 = (m + 1) / 3, n2 = m / 3;
  const u64 m12 = n0 + n2;
  const u32 dummy = n0 > n1 ? 1u : 0u;
  const u64 n12 = m12 - dummy;  // real sample suffixes
  const int bsym = bits_of(max_sym);
  Dc3Level L;
  if (!level_alloc(c, depth, 0, m12, &L.child) || !level_alloc(c, depth, 1, m12, &L.tmp) ||
      !level_alloc(c, depth, 2, m + 3, &L.rankp) || !level_alloc(c, depth, 3, n12, &L.byrank))
    return SA_ENOMEM;
  launch_fill_u32(L.rankp, m + 3, 0, s);
  const Bufs full = full_bufs(c);
  const u32 grid12 = stream_grid(c, m12, 256);

  // Step 2: sort the sample by triples and name them (head ranks). The re-rank
  // in its first-round form writes the names to `child` (its ISA argument),
  // unique ones' sample indices to tmp[name - 1], and counts the others.
  {
    Tracer t(c, s, SA_KERNEL_PACK_TEXT, double(m12) * 24.0);
    if (3 * bsym <= 64)
      hipLaunchKernelGGL((dc3_pack_kernel<T, 1>), dim3(grid12), dim3(256), 0, s, str, m12, n0,
                         bsym, full.kA, full.vA);
    else
      hipLaunchKernelGGL((dc3_pack_kernel<T, 2>), dim3(grid12), dim3(256), 0, s, str, m12, n0,
                         bsym, full.kA, full.vA);
  }
  const int word_bits = 3 * bsym <= 64 ? 3 * bsym : 2 * bsym;
  run_sort(c, full, m12, npass_for(c, word_bits), 1, 0, s);
  RerankArgs a = single_args(m12, m12, 0, kRerankScatterIsa);
  if (3 * bsym > 64) {
    // Run names of the low word, then the high word x[p] sorted stably with
    // them as tie words.
    u64* pk = reinterpret_cast<u64*>(c->act_idx);
    RerankArgs lo = single_args(m12, m12, 0, kRerankPairOut);
    lo.pair_out = pk;
    run_rerank(c, full, lo, L.tmp, m12, m12, s);
    hipLaunchKernelGGL((dc3_pack_hi_kernel<T>), dim3(grid12), dim3(256), 0, s, str, c->ctl, n0, pk,
                       full.kA);
    begin_sort(c, m12, &c->ctl->count, nullptr, npass_for(c, bsym), true, s);
    sort_passes(c, full, m12, npass_for(c, bsym), 0, kMaxRounds, m12, s);
    launch_quad_permute(c->ctl, c->plan, pk, full.vA, full.vB, c->counters, grid12, s);
    a.tie = 1;
  }
  {
    Tracer t(c, s, SA_KERNEL_RERANK, double(m12) * 16.0);
    const u32 grid = u32(std::min<u64>(std::max<u64>(1, ceil_div(m12, kRerankTile)),
                                       u64(c->num_cus) * rerank_wgs_per_cu(a.tie != 0)));
    launch_rerank_compact(full.kA, full.kB, full.vA, full.vB, c->plan, a, c->ctl, L.child, L.tmp,
                          c->act_idx, nullptr, c->act_rank, c->counters, grid, s);
  }
  sa_status st = readback(c, s);
  if (st != SA_OK) return st;
  const u64 nonunique = c->h_counters[kCtrActive];
  const u32* sa12 = L.tmp;
  if (nonunique > 0) {
    // Equal triples: the sample's order is the suffix order of the names.
    if (!level_alloc(c, depth, 4, m12, &L.childsa)) return SA_ENOMEM;
    st = dc3_level<u32>(c, L.child, m12, 0, m12, L.childsa, nullptr, depth + 1, s);
    if (st != SA_OK) return st;
    sa12 = L.childsa;
  }
  hipLaunchKernelGGL(dc3_ranks_kernel, dim3(scatter_grid(c, m12)), dim3(256), 0, s, sa12, m12, n0,
                     m, dummy, L.rankp, L.byrank, c->counters);

  // Step 3: the mod-0 suffixes by (x[i], rank(i + 1)).
  const int brank = std::max(1, bits_of(n12));
  {
    Tracer t(c, s, SA_KERNEL_PACK_TEXT, double(n0) * 16.0);
    hipLaunchKernelGGL((dc3_pack_s0_kernel<T>), dim3(stream_grid(c, n0, 256)), dim3(256), 0, s,
                       str, n0, L.rankp, brank, full.kA, full.vA);
  }
  run_sort(c, full, n0, npass_for(c, bsym + brank), 1, 0, s);

  // Step 4: comparison records, merge-path splits, merge by tiles.
  const u64 ntiles = ceil_div(m, u64(kDc3Tile));
  if (!level_alloc(c, depth, 5, n0, &L.rec0) || !level_alloc(c, depth, 6, n12, &L.rec12) ||
      !level_alloc(c, depth, 7, n0, &L.pos0) || !level_alloc(c, depth, 8, ntiles + 1, &L.split))
    return SA_ENOMEM;
  {
    // Position in; two characters and two ranks gathered; a 16-byte record out.
    Tracer t(c, s, SA_KERNEL_OTHER, double(m) * 32.0);
    hipLaunchKernelGGL((dc3_records_kernel<T>), dim3(stream_grid(c, m, 256)), dim3(256), 0, s,
                       str, n0, n12, full.vA, full.vB, c->plan, L.rankp, L.byrank, L.rec0, L.pos0,
                       L.rec12);
    hipLaunchKernelGGL(dc3_partition_kernel, dim3(u32(ceil_div(ntiles + 1, 256))), dim3(256), 0,
                       s, L.rec0, L.rec12, L.byrank, n0, n12, u64(kDc3Tile), ntiles, L.split);
  }
  {
    // Records and positions in, the suffix array out.
    Tracer t(c, s, SA_KERNEL_OTHER, double(m) * 24.0);
    hipLaunchKernelGGL(dc3_merge_tile_kernel, dim3(u32(ntiles)), dim3(256), 0, s, L.rec0, L.pos0,
                       L.rec12, L.byrank, L.split, n0, n12, sa, c->counters);
  }
  if (rank_out)
    hipLaunchKernelGGL(dc3_rank_out_kernel, dim3(stream_grid(c, m, 256)), dim3(256), 0, s,
                       L.rankp, m, rank_out);
  // The arrays stay with the context; the top level checks the error flags.
  return depth == 0 ? readback(c, s) : SA_OK;
}

sa_status dc3_names(sa_ctx* c, const u32* x, u64 m, u64 max_sym, u32* sa, u32 depth,
                    hipStream_t s) {
  return dc3_level<u32>(c, x, m, 0, max_sym, sa, nullptr, depth, s);
}

sa_status build_dc3(sa_ctx* c, const u8* text, u64 n, u32* d_sa, u32* d_rank12, hipStream_t s) {
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
  return dc3_level<u8>(c, text, n, 1, 256, d_sa, d_rank12, 0, s);
}

}  // namespace drv

using namespace drv;

extern "C" {

sa_status sa_build_dc3(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t* d_sa,
                       uint32_t* d_rank12, void* stream) {
  if (!ctx) return SA_EINVAL;
  const sa_status st = build_dc3(ctx, d_text, n, d_sa, d_rank12, static_cast<hipStream_t>(stream));
  settle_trace(ctx, st);
  return st;
}

}  // extern "C"
