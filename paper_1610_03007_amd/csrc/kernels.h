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
// counters hold sigma, the code width w = bits(sigma) and c = floor(64 / w).
void launch_byte_presence(const u8* text, u64 n, u32* present, hipStream_t s);
void launch_alphabet_codes(const u32* present, u16* code, u64* counters, hipStream_t s);

// Round-0 keys: key[i] = c codes of T[i, i+c) (0 past the end), w bits each,
// first character most significant.
void launch_pack_text(const u8* text, u64 n, const u16* code, const u64* counters, u64* keys,
                      hipStream_t s);

// Round >= 1 keys: key[p] = (rank[p] << b) | (idx[p] + h < n ? isa[idx[p] + h] : 0);
// vals[p] = idx[p].
void launch_pack_pairs(const u32* act_idx, const u32* act_rank, u64 count, u64 n, u64 h, int b,
                       const u32* isa, u64* keys, u32* vals, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs held in buffer A, 8-bit digits over
// the low `npass` digits. hist must hold kMaxPasses * kRadix zeroed words and the
// pass ticket counters must be zero. Which buffer ends up sorted is recorded in
// plan->final_buf. With vals_present == 0 the values are generated (input index).
void launch_radix_histogram(const u64* keys, u64 count, int npass, u64* hist, hipStream_t s);
void launch_radix_plan(const u64* hist, u64 count, int npass, int vals_present, SortPlan* plan,
                       hipStream_t s);
void launch_onesweep_pass(u64* keysA, u64* keysB, u32* valsA, u32* valsB, u64 count, int pass,
                          const SortPlan* plan, u64* status, u64* counters, u32 gen,
                          hipStream_t s);

// Re-rank the sorted active set, scatter the ISA, finalize unique suffixes into
// the SA and compact the survivors. b = bits of the second rank (0 in round 0,
// where every element starts with rank 1).
void launch_rerank_compact(const u64* keysA, const u64* keysB, const u32* valsA,
                           const u32* valsB, const SortPlan* plan, u64 count, u64 n, int b,
                           u32* isa, u32* sa_out, u32* act_idx, u32* act_rank, u64* st_head,
                           u64* st_grp, u64* st_surv, u64* counters, u32 gen, hipStream_t s);

inline u64 ceil_div(u64 a, u64 b) { return (a + b - 1) / b; }

}  // namespace sa
