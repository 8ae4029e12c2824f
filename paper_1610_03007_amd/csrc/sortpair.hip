// Prefix doubling with discarding by sorting (Section 2.1, Alg. 5 with the
// comparator of Eq. 1 and the helper functions of Alg. 6): the variant that
// needs no inverse suffix array, for a text spread over devices where a random
// read of ISA[i + h] would cross devices. Each round works on the items P =
// (position, name, unique flag):
//
//   1. sort P by (i mod h, i div h), so that suffix i + h follows suffix i
//      whenever both are present (the comparator, as a radix key);
//   2. one scan: a non-unique item takes the name of its successor if that is
//      suffix i + h, else the sentinel 0; a unique item is kept for the next
//      round only if the two items before it are both non-unique (one of them
//      may still need its name), otherwise its name is final: SA[name - 1] = i;
//   3. sort the non-unique items by name pair and rename them (old name plus
//      the offset of the run of equal pairs in the group of equal old names),
//      writing them with their new unique flags as the next round's items,
//      after the kept ones.
//
// The loop ends when no item is non-unique; every item is then discarded.

#include "driver.h"

namespace sa {

// Step 2 over the ctl->count sorted items (buffer plan->final_buf): pairs go
// to (ikeys, ivals) as (name << b | next name, position), kept unique items to
// (ukeys, uvals) keyed for the next offset h2, both compacted with one atomic
// per wave into counters[kCtrPairI] / counters[kCtrPairU] (zero on entry).
__global__ __launch_bounds__(256) void npairs_kernel(
    const u64* __restrict__ kA, const u64* __restrict__ kB, const u32* __restrict__ vA,
    const u32* __restrict__ vB, const SortPlan* __restrict__ plan,
    const SortCtl* __restrict__ ctl, u64 n, u64 h, u64 q, int b, u64 h2, u64 q2,
    u64* __restrict__ ikeys, u32* __restrict__ ivals, u64* __restrict__ ukeys,
    u32* __restrict__ uvals, u32* __restrict__ sa, u64* __restrict__ counters) {
  const u64 count = ctl->count;
  const u32 fb = plan->final_buf;
  const u64* keys = fb ? kB : kA;
  const u32* vals = fb ? vB : vA;
  const int lane = threadIdx.x & (kWave - 1);
  const u64 lt = (u64(1) << lane) - 1;
  const u64 wpb = blockDim.x / kWave;
  const u64 stride = u64(gridDim.x) * wpb * kWave;
  bool bad = false;
  // Every lane of a wave runs the same iterations (ballots below).
  for (u64 base = (u64(blockIdx.x) * wpb + threadIdx.x / kWave) * kWave; base < count;
       base += stride) {
    const u64 p = base + lane;
    const bool valid = p < count;
    const u64 key = valid ? keys[p] : 0;
    const u32 r = valid ? vals[p] : 0;
    const bool uniq = (key & kUniqueBit) != 0;
    const u64 i = opk_pos(key & ~kUniqueBit, h, q);
    bool to_i = false, keep = false;
    u64 ikey = 0;
    if (valid && i >= n) {
      bad = true;
    } else if (valid && !uniq) {
      u32 r1 = 0;
      if (p + 1 < count && opk_pos(keys[p + 1] & ~kUniqueBit, h, q) == i + h) r1 = vals[p + 1];
      ikey = (u64(r) << b) | u64(r1);
      to_i = true;
    } else if (valid) {
      keep = p >= 2 && !(keys[p - 1] & kUniqueBit) && !(keys[p - 2] & kUniqueBit);
      if (!keep) {
        if (r == 0 || r > n)
          bad = true;
        else
          sa[r - 1] = u32(i);
      }
    }
    const u64 bi = __ballot(to_i), bu = __ballot(keep);
    unsigned long long ib = 0, ub = 0;
    if (lane == 0) {
      if (bi)
        ib = atomicAdd(reinterpret_cast<unsigned long long*>(counters + kCtrPairI),
                       (unsigned long long)__popcll(bi));
      if (bu)
        ub = atomicAdd(reinterpret_cast<unsigned long long*>(counters + kCtrPairU),
                       (unsigned long long)__popcll(bu));
    }
    ib = __shfl(ib, 0, kWave);
    ub = __shfl(ub, 0, kWave);
    if (to_i) {
      const u64 o = u64(ib) + u64(__popcll(bi & lt));
      if (o < count) {
        ikeys[o] = ikey;
        ivals[o] = u32(i);
      } else {
        bad = true;
      }
    }
    if (keep) {
      const u64 o = u64(ub) + u64(__popcll(bu & lt));
      if (o < count) {
        ukeys[o] = opk_key(i, h2, q2) | kUniqueBit;
        uvals[o] = r;
      } else {
        bad = true;
      }
    }
  }
  if (bad)
    atomicOr(reinterpret_cast<unsigned long long*>(counters + kCtrError),
             (unsigned long long)kErrBounds);
}

}  // namespace sa

namespace drv {

void free_pair_workspace(sa_ctx* c) {
  for (int j = 0; j < 3; ++j) {
    (void)hipFree(c->pair_k[j]);
    (void)hipFree(c->pair_v[j]);
    c->pair_k[j] = nullptr;
    c->pair_v[j] = nullptr;
  }
  c->pair_cap = 0;
}

// Three item buffers: two for the comparator sort's ping-pong, one that
// receives the next round's items while the sorted ones are read.
sa_status ensure_pair_workspace(sa_ctx* c, u64 n) {
  if (n <= c->pair_cap) return SA_OK;
  free_pair_workspace(c);
  const u64 cap = std::max<u64>(n, 1 << 16);
  for (int j = 0; j < 3; ++j)
    if (!dev_alloc(&c->pair_k[j], cap) || !dev_alloc(&c->pair_v[j], cap)) {
      free_pair_workspace(c);
      return SA_ENOMEM;
    }
  c->pair_cap = cap;
  return SA_OK;
}

sa_status build_sortpair(sa_ctx* c, const u8* text, u64 n, u32* d_sa, u64* h_counts,
                         u32 max_counts, hipStream_t s) {
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
  st = ensure_pair_workspace(c, n);
  if (st != SA_OK) return st;

  // Round 0: names of c-character prefixes (as sa_build's round 0).
  const Bufs full = full_bufs(c);
  {
    Tracer t(c, s, SA_KERNEL_OTHER, 0);
    launch_fill_u64(c->counters, kCtrCount, 0, s);
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
  st = readback(c, s);  // the round-0 width c fixes the first offset
  if (st != SA_OK) return st;
  sa_build_info& info = c->info;
  info.sigma = u32(c->h_counters[kCtrSigma]);
  info.code_bits = u32(c->h_counters[kCtrCodeBits]);
  info.chars0 = u32(c->h_counters[kCtrChars]);
  info.rounds = 1;
  info.active[0] = n;
  info.key_bits[0] = info.code_bits * info.chars0;
  info.passes_run[0] = passes_run(c, 0, npass0);
  const u64 c0 = info.chars0;
  const int b = bits_of(n);
  int A = 0, B = 1, W = 2;
  {
    // Every suffix becomes an item of round 1 (offset c0), in name order.
    RerankArgs a = single_args(n, n, 0, kRerankEmit);
    a.emit_keys = c->pair_k[A];
    a.emit_vals = c->pair_v[A];
    a.emit_base = c->counters + kCtrPairU;  // 0
    a.emit_h = c0;
    a.emit_q = ceil_div(n, c0);
    run_rerank(c, full, a, d_sa, n, n, s);
  }
  u64 pcount = n;
  u64 h = c0;
  for (u32 k = 1;; ++k) {
    if (k >= u32(SA_MAX_ROUNDS)) return SA_EDEVICE;  // cannot happen for n < 2^32
    const u64 q = ceil_div(n, h);
    const u64 h2 = 2 * h, q2 = ceil_div(n, h2);
    const int npass_p = npass_for(c, std::max(1, bits_of(h * q - 1)));
    const int npass_i = npass_for(c, 2 * b);
    const Bufs pb{c->pair_k[A], c->pair_k[B], c->pair_v[A], c->pair_v[B]};
    run_sort(c, pb, pcount, npass_p, 1, int(k), s);
    {
      Tracer t(c, s, SA_KERNEL_PACK_PAIRS, double(pcount) * 24.0);
      launch_fill_u64(c->counters + kCtrPairI, 2, 0, s);
      const u32 grid = scatter_grid(c, pcount);  // discarded suffixes scatter into SA
      hipLaunchKernelGGL(npairs_kernel, dim3(grid), dim3(256), 0, s, pb.kA, pb.kB, pb.vA, pb.vB,
                         c->plan, c->ctl, n, h, q, b, h2, q2, c->keysA, c->valsA, c->pair_k[W],
                         c->pair_v[W], d_sa, c->counters);
    }
    // Tracing attributes bytes per launch, so it reads the pair count back.
    u64 traced = pcount;
    if (c->trace) {
      st = readback(c, s);
      if (st != SA_OK) return st;
      traced = c->h_counters[kCtrPairI];
    }
    // The non-unique items, by name pair; renamed into the next round's items.
    begin_sort(c, pcount, c->counters + kCtrPairI, nullptr, npass_i, true, s);
    sort_passes(c, full, pcount, npass_i, 1, int(k) + kPlanRowSecond, traced, s);
    {
      RerankArgs a = single_args(pcount, n, b, kRerankEmit);
      a.emit_keys = c->pair_k[W];
      a.emit_vals = c->pair_v[W];
      a.emit_base = c->counters + kCtrPairU;
      a.emit_h = h2;
      a.emit_q = q2;
      run_rerank(c, full, a, d_sa, pcount, traced, s);
    }
    st = readback(c, s);
    if (st != SA_OK) return st;
    const u64 ni = c->h_counters[kCtrPairI], nu = c->h_counters[kCtrPairU];
    if (ni + nu > pcount) return SA_EDEVICE;
    if (k < max_counts && h_counts) {
      u64* row = h_counts + 4 * size_t(k - 1);
      row[0] = pcount;
      row[1] = ni;
      row[2] = pcount - ni - nu;
      row[3] = nu;
    }
    info.active[k] = pcount;
    info.key_bits[k] = u32(2 * b);
    info.passes_run[k] = passes_run(c, int(k), npass_p) +
                         passes_run(c, int(k) + kPlanRowSecond, npass_i);
    info.rounds = 1 + k;
    info.prefix_len = c0 << k;
    if (ni == 0) {
      // No non-unique item: every item was discarded, so the SA is complete.
      return nu == 0 ? SA_OK : SA_EDEVICE;
    }
    pcount = ni + nu;
    h = h2;
    const int oa = A, ob = B;
    A = W;
    B = oa;
    W = ob;
  }
}

}  // namespace drv

using namespace drv;

extern "C" {

sa_status sa_build_sorted_pairs(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma,
                                uint32_t* d_sa, uint64_t* h_counts, uint32_t max_rounds,
                                void* stream) {
  if (!ctx) return SA_EINVAL;
  if (sigma == 0 || sigma > 256) return SA_EINVAL;
  ctx->sigma_hint = sigma;
  const sa_status st = build_sortpair(ctx, d_text, n, d_sa, h_counts, max_rounds + 1,
                                      static_cast<hipStream_t>(stream));
  ctx->sigma_hint = 0;
  settle_trace(ctx, st);
  return st;
}

}  // extern "C"
