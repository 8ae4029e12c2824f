// Host-side launchers for the gfx950 suffix-array kernels (sa_kernels.hip).
#pragma once

#include "common.h"

namespace sa {

// Fills `count` 64-bit words with `value`.
void launch_fill_u64(u64* p, u64 count, u64 value, hipStream_t s);
// sa[0] = 0 (text of length one).
void launch_set_zero_u32(u32* p, hipStream_t s);

// Alphabet reduction: present[256] must be zero on entry. Afterwards code[b] is
// 1 + (number of present bytes below b) for every present byte b, and the
// counters hold sigma, the code width w = bits(sigma) and c <= floor(64 / w).
void launch_byte_presence(const u8* text, u64 n, u32* present, hipStream_t s);
// The key holds idbits + c * w bits (idbits = text-id bits of a batch, else 0).
// With trim != 0, c is lowered so that the key fills whole 8-bit radix digits.
void launch_alphabet_codes(const u32* present, u16* code, u64* counters, int trim, int idbits,
                           hipStream_t s);

// Round-0 keys: key[i] = c codes of T[i, i+c) (0 past the end), w bits each,
// first character most significant.
void launch_pack_text(const u8* text, u64 n, const u16* code, const u64* counters, u64* keys,
                      hipStream_t s);

// Round >= 1 keys: key[p] = (rank[p] << b) | (idx[p] + h < n ? isa[idx[p] + h] : 0);
// vals[p] = idx[p].
void launch_pack_pairs(const u32* act_idx, const u32* act_rank, u64 count, u64 n, u64 h, int b,
                       const u32* isa, u64* keys, u32* vals, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs held in buffer A, 8-bit digits over
// the low `npass` digits. Geometry: tiles of `tile` pairs grouped into chunks of
// 2^ct_log2 tiles, nchunks = number of non-empty chunks (<= kChunks).
struct SortGeom {
  u64 count;
  u32 tile;
  u32 ct_log2;
  u32 nchunks;
};
// hist_in [kMaxPasses][kChunks][kRadix] must be zero on entry, and
// counters[kCtrKeyOr], counters[kCtrKeyNot] zero. Receives the per-chunk
// counts of digits 0 and 1 and the OR of the keys and of their complements.
void launch_radix_histogram(const u64* keys, const SortGeom& geo, u32* hist_in, u64* counters,
                            hipStream_t s);
// Skipped passes (constant digits, from the two ORs) and the buffer schedule.
// With vals_present == 0 the first sweep generates the values (input index).
void launch_radix_plan(const u64* counters, int npass, int vals_present, SortPlan* plan,
                       hipStream_t s);
// Per-chunk counts of the first sweep's digit when it is above digit 1 (a
// no-op otherwise, decided on the device from the plan).
void launch_radix_histogram_first(const u64* keys, const SortGeom& geo, const SortPlan* plan,
                                  u32* hist_in, hipStream_t s);
// One sweep. hist_run [kMaxPasses][kChunks][kRadix] and tickets
// [kMaxPasses][kChunks] must be zero before the first sweep of a sort. `items`
// per thread (8, 12, 16, 20 or 24 with 256-thread workgroups; 4, 8 or 12 with
// 512) and `block` must match geo.tile = block * items.
// `grid` persistent workgroups (a multiple of geo.nchunks).
// Workgroups of the sweep of this shape that one CU holds at once (the
// runtime's occupancy query: registers and LDS), or 0 if the query fails.
int onesweep_wgs_per_cu(int items, int block, bool table);
// table: digit matching through an LDS table (true) or through ballots (false);
// both give the same result.
void launch_onesweep_pass(u64* keysA, u64* keysB, u32* valsA, u32* valsB, const SortGeom& geo,
                          int pass, const SortPlan* plan, const u32* hist_in, u32* hist_run,
                          u32* tickets, u64* status, u64* counters, u32 gen, int items,
                          int block, bool table, u32 grid, hipStream_t s);

// Re-rank the sorted active set, scatter the ISA, finalize unique suffixes into
// the SA and compact the survivors.
// mode: kRerankScatterIsa writes ISA[text position] = new rank for every element
// (in rounds after a text's round 0, only where the rank changed);
// kRerankIsaOnly, with it, writes nothing else (no SA entries, no survivors,
// no survivor count): the eager ISA after a round 0 that ran without it.
constexpr int kRerankScatterIsa = 1;
constexpr int kRerankIsaOnly = 4;
// Key layout of the sorted set:
//   group     = key >> gshift (64: one group, round 0 of a single text)
//   old rank  = (key >> rshift) & rmask (rmask 0: every element has rank 1)
//   text id   = key >> idshift in multi-text mode; ranks and positions are
//               then local to that text, SA and ISA are addressed at
//               tbase[t] + local, survivors go to act_ti as (t << 32) | local
//               instead of act_idx.
struct RerankArgs {
  u64 count;
  u64 n;
  int gshift;
  int rshift;
  u64 rmask;
  int idshift;
  int mode;
  // Multi-text mode (tbase set): text t = key >> idshift starts at tbase[t] in
  // the SA / ISA arenas and has tlen[t] suffixes; texts with tround0[t] set
  // carry round-0 keys (one group per text, every rank 1).
  const u64* tbase;
  const u64* tlen;
  const u8* tround0;
};
void launch_rerank_compact(const u64* keysA, const u64* keysB, const u32* valsA,
                           const u32* valsB, const SortPlan* plan, const RerankArgs& args,
                           u32* isa, u32* sa_out, u32* act_idx, u64* act_ti, u32* act_rank,
                           u64* counters, hipStream_t s);

// ISA after round 0. Eager: the round-0 re-rank again, with kRerankIsaOnly.
// Lazy: survivors scattered from the active list and marked in the live-position
// bitmap; other names resolved on demand by a binary search in the round-0
// sorted keys `keys0`.
void launch_isa_scatter_list(const u32* idx, const u32* rank, u64 count, u64 n, u32* isa,
                             u32* live, hipStream_t s);
// Lazy ISA: sample[i] = keys0[i * n / kLazySamples] of the round-0 sorted keys,
// the first step of every round-0 name search.
constexpr u32 kLazySamples = 4096;
void launch_lazy_sample(const u64* keys0, u64 n, u64* sample, hipStream_t s);
void launch_pack_pairs_lazy(const u32* act_idx, const u32* act_rank, u64 count, u64 n, u64 h,
                            int b, const u32* isa, const u8* text, const u16* code,
                            const u64* counters, const u64* keys0, const u64* sample,
                            const u32* live, u64* keys, u32* vals, hipStream_t s);
void launch_isa_complete(u32* isa, u64 n, const u8* text, const u16* code, const u64* counters,
                         const u64* keys0, const u64* sample, const u32* live, hipStream_t s);
void launch_fill_u32(u32* p, u64 count, u32 value, hipStream_t s);

__host__ __device__ inline u64 ceil_div(u64 a, u64 b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Multi-text engine (batched builds and the server): per-text tables.
struct TextTab {
  u64* base;     // [slots] first position of the text in the text / SA / ISA arenas
  u64* len;      // [slots] text length
  u16* code;     // [slots][256] character codes 1..sigma_t (0: absent)
  u32* present;  // [slots][8] bitmap of the bytes present (zero between uses)
  u32* wc;       // [slots] code width w | characters per round-0 key c << 16
  u64* h;        // [slots] doubling offset of the text's next round
  u8* round0;    // [slots] 1 while the text's elements carry round-0 keys
  u32* surv;     // [slots] survivors of the text after the last round
};
// Texts entering round 0 this round: text slot t[i] (i < m), whose elements go
// to positions out[i] .. out[i] + len of the merged key array; chunk0[i] is the
// first of its ceil(len / kNewChunk) chunks (chunk0[m] = total chunks).
constexpr int kNewChunk = 2048;
struct NewList {
  const u32* t;
  const u64* out;
  const u64* chunk0;
  u32 m;
  u64 chunks;
};
void launch_multi_presence(const u8* arena, TextTab tab, NewList nl, hipStream_t s);
// c = characters per round-0 key: floor((64 - idbits) / w), trimmed to whole
// 8-bit digits of the full key when trim != 0. Clears the presence bitmaps.
void launch_multi_codes(TextTab tab, NewList nl, int idbits, int trim, hipStream_t s);
// Round-0 keys: (t << idshift) | c codes of text t from local position i (0 past
// its end); values = i.
void launch_multi_pack0(const u8* arena, TextTab tab, NewList nl, int idshift, u64* keys,
                        u32* vals, hipStream_t s);
// Later-round keys for survivors (t, i, r): (t << idshift) | (r << b) |
// (i + h_t < n_t ? ISA[base_t + i + h_t] : 0); values = i.
// Batched build with a lazy ISA after round 0 (see sa_kernels.hip).
void launch_multi_isa_scatter_list(const u64* act_ti, const u32* act_rank, const u64* count_ptr,
                                   u64 bound, TextTab tab, u32* isa, u32* live, hipStream_t s);
void launch_multi_pack_pairs_lazy(const u64* act_ti, const u32* act_rank, u64 count, TextTab tab,
                                  int b, int idshift, const u32* isa, const u32* live,
                                  const u8* arena, const u64* keys0, u64* keys, u32* vals,
                                  hipStream_t s);
void launch_multi_pack_pairs(const u64* act_ti, const u32* act_rank, u64 count, TextTab tab,
                             int b, int idshift, const u32* isa, u64* keys, u32* vals,
                             hipStream_t s);
// surv[t] += number of survivors of text t among act_ti[0 .. *count_ptr)
// (surv must be cleared before; bound >= *count_ptr sizes the launch).
void launch_multi_count_survivors(const u64* act_ti, const u64* count_ptr, u64 bound, u32* surv,
                                  hipStream_t s);

}  // namespace sa
