// Shared definitions for the gfx950 suffix-array kernels and their host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sa {

typedef uint64_t u64;
typedef uint32_t u32;
typedef uint16_t u16;
typedef uint8_t u8;

constexpr int kWave = 64;  // CDNA wavefront width

// ---------------------------------------------------------------------------
// Decoupled look-back status words (single-pass scans across workgroups).
//
// A 64-bit word holds [generation:22 | flag:2 | value:40]. The generation is a
// launch counter kept by the host, so a status array never has to be cleared
// between launches: a word written by an older launch reads as "not ready".
// flag 1 = aggregate of this tile only, flag 2 = inclusive prefix.
constexpr u64 kStatusValueBits = 40;
constexpr u64 kStatusValueMask = (u64(1) << kStatusValueBits) - 1;
constexpr u32 kFlagAggregate = 1;
constexpr u32 kFlagPrefix = 2;
constexpr u32 kGenMask = (1u << 22) - 1;

__host__ __device__ inline u64 status_pack(u32 gen, u32 flag, u64 value) {
  return (u64(gen & kGenMask) << 42) | (u64(flag) << 40) | (value & kStatusValueMask);
}
__host__ __device__ inline u32 status_gen(u64 s) { return u32(s >> 42) & kGenMask; }
__host__ __device__ inline u32 status_flag(u64 s) { return u32(s >> 40) & 3u; }
__host__ __device__ inline u64 status_value(u64 s) { return s & kStatusValueMask; }

// Bounded wait: a look-back that does not see its predecessor within this many
// polls raises the error flag and gives up, so a kernel always terminates.
constexpr u32 kSpinLimit = 1u << 24;

// Error flag bits reported back to the host.
constexpr u32 kErrLookbackTimeout = 1u;
constexpr u32 kErrBounds = 2u;  // an index fell outside its array; the write was dropped

__device__ inline u64 load_status(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_status(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Radix sort plan, computed on the device from the up-front digit histograms.
// Digits are kRadixBits wide by default; a tuning may choose any width in
// [kRadixBitsMin, kRadixBitsMax]. Per-digit arrays are sized for the widest
// digit, per-pass arrays for the narrowest.
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kRadixBitsMin = 6;
constexpr int kRadixBitsMax = 9;
constexpr int kRadixMax = 1 << kRadixBitsMax;
constexpr int kMaxPasses = (64 + kRadixBitsMin - 1) / kRadixBitsMin;
// Passes of rb-bit digits that cover `bits` key bits.
__host__ __device__ constexpr int passes_for(int bits, int rb) { return (bits + rb - 1) / rb; }

struct SortPlan {
  u32 skip[kMaxPasses];             // pass p is skipped (its digit is constant)
  u32 src[kMaxPasses];              // buffer pass p reads (0 = A, 1 = B)
  u32 iota[kMaxPasses];             // pass p generates values = input index
  u32 final_buf;                    // buffer that holds the sorted output
  u32 first_run;                    // first pass that runs
  int next_run[kMaxPasses];         // next pass that runs after p, or -1
};

// Each sweep splits its tiles into up to kChunks contiguous chunks with
// independent look-back chains. The digit counts of every chunk are known
// before the sweep starts (for the first sweep from the up-front histogram,
// for later ones accumulated by the sweep before), so a chunk's first tile
// never waits on another chunk; summed over the chunks they also give the
// sweep its global digit offsets.
constexpr int kChunks = 32;
static_assert(kChunks % 8 == 0, "chunk counts are read eight at a time");

// Sweep geometry of a sort of `count` pairs in tiles of `tile`: the tiles are
// grouped into chunks of `per` = ceil(tiles / kChunks) tiles, so that kChunks
// chunks cover a large input (nchunks of them non-empty). With the persistent
// sweep's workgroup b on chunk b mod nchunks and workgroups dealt to the 8 XCDs
// in turn, 32 chunks keep each chunk's tiles on one XCD, whose L2 then joins the
// partial lines that neighbouring tiles write at the ends of their digit runs
// (a power-of-two chunk size left the 4.46e9-pair batch with 17 chunks spread
// over every XCD, and its sweep 6% slower). chunk_of(t) = t / per by a
// multiply-high with magic = ceil(2^32 / per) and one correction step. Host and
// device derive it alike.
struct SortGeom {
  u64 count;
  u32 tile;
  u32 per;
  u32 nchunks;
  u64 magic;
};
__host__ __device__ inline u32 chunk_of(const SortGeom& g, u32 t) {
  u32 q = u32((u64(t) * g.magic) >> 32);  // t / per or one more
  if (u64(q) * g.per > t) --q;
  return q;
}
// Sort-based pairing (Eq. 1): position i is keyed (i mod h) * q + (i div h)
// with q = ceil(n / h), so that positions ordered by key are ordered by
// residue modulo h, then by quotient: suffix i + h directly follows suffix i
// when both are present. Keys stay below h * q <= n + h - 1.
// (32-bit division when the operands fit: 64-bit division is a long
// instruction sequence on the GPU.)
__host__ __device__ inline u64 opk_key(u64 i, u64 h, u64 q) {
  if ((i | h) >> 32 == 0) return u64(u32(i) % u32(h)) * q + u32(i) / u32(h);
  return (i % h) * q + i / h;
}
__host__ __device__ inline u64 opk_pos(u64 key, u64 h, u64 q) {
  if ((key | q) >> 32 == 0) return u64(u32(key) % u32(q)) * h + u32(key) / u32(q);
  return (key % q) * h + key / q;
}

__host__ __device__ inline SortGeom sort_geom(u64 count, u32 tile) {
  SortGeom g;
  g.count = count;
  g.tile = tile;
  u64 tiles = (count + tile - 1) / tile;
  if (tiles < 1) tiles = 1;
  const u64 per = (tiles + kChunks - 1) / kChunks;
  g.per = u32(per);
  g.nchunks = u32((tiles + per - 1) / per);
  g.magic = ((u64(1) << 32) + per - 1) / per;
  return g;
}

// Control words of the current sort, in device memory. sort_begin_kernel sets
// them (from a count the host passes, or from a device counter such as the
// survivor count of the last re-rank) and every later kernel of the sort and
// of the re-rank reads them instead of taking the count as an argument, so
// that a captured round replays with unchanged launch arguments. A count of 0
// makes every kernel of the round return at once.
struct SortCtl {
  u64 count;     // pairs in the sort
  u32 gen_base;  // look-back generation of pass 0 (pass p uses gen_base + p)
  u32 gen_next;  // first generation not used yet
  u32 dense;     // 1: a dense round (every suffix, keys built in position order)
  u32 reserved;
};

// Doubling rounds of one text run ahead of the host: the index and offset of
// the round in progress, and a log the host reads back.
constexpr int kMaxRounds = 64;
struct RoundCtl {
  u32 round;                // later rounds started (round 0 not counted)
  u32 reserved;
  u64 h;                    // doubling offset of the round in progress
  u64 dense;                // bit k: round k was dense
  u64 active[kMaxRounds];   // suffixes sorted in round k (k >= 1)
};
// Plan log: the flags of the sort of round k (kPlanLogWords words per round):
// skip[kMaxPasses] | src[kMaxPasses] | iota[kMaxPasses] | final buffer. Row
// k + kPlanRowSecond holds the second sort of a quadrupling round k (the high
// word of its two-word keys).
constexpr int kPlanLogWords = 3 * kMaxPasses + 1;
constexpr int kPlanRowSecond = kMaxRounds + 1;
constexpr int kPlanLogRows = 2 * kPlanRowSecond;
// log_row values that name a row through the round index on the device.
constexpr int kLogRowRound = -1;         // row rc->round
constexpr int kLogRowRoundSecond = -2;   // row rc->round + kPlanRowSecond

// Workgroup and tile shapes.
constexpr int kSortBlock = 256;          // the smaller sweep workgroup (one thread per digit)
constexpr int kSortBlockDefault = 512;   // default sweep shape: 512 threads x 8 items
constexpr int kSortItemsDefault = 8;
constexpr int kSortTileMin = 2048;       // smallest tile (512 x 4); status arrays are sized for it
constexpr int kHistBlock = 256;
// Staged ISA writes of a re-rank over a large active set: (position, name)
// pairs grouped by position bucket (kStageBuckets equal ranges of the text)
// and then written one bucket after the other, so that the writes in flight
// fall in one bucket's stretch of the ISA instead of all of it.
constexpr int kStageBuckets = 256;
constexpr u32 kStageMaxWgs = 1024;               // re-rank workgroups with a count row
constexpr u64 kStageMinCount = u64(1) << 22;     // active elements (read on the device)
constexpr u64 kStageMinN = u64(1) << 26;         // text length (ISA of 256 MiB)
constexpr u64 kStageSkip = ~u64(0);              // staged entry: name unchanged

constexpr int kRerankBlock = 256;
constexpr int kRerankRows = 8;  // rows of 64 elements per wave
constexpr int kRerankTile = kRerankBlock * kRerankRows;  // 2048 elements

// Device-side 64-bit counters shared by one build (slot indices).
enum CounterSlot : int {
  kCtrSortTiles = 0,                 // kMaxPasses slots: tile tickets per pass
  kCtrKeyOr = kMaxPasses,            // OR of the keys being sorted
  kCtrKeyNot = kMaxPasses + 1,       // OR of their complements (a digit varies where both are set)
  kCtrActive = kMaxPasses + 2,       // survivors written by the last re-rank (atomic sum)
  kCtrError = kMaxPasses + 3,        // error bits (kErr*)
  kCtrSigma = kMaxPasses + 4,        // distinct bytes in the text
  kCtrCodeBits = kMaxPasses + 5,     // w: bits per character code
  kCtrChars = kMaxPasses + 6,        // c: characters packed in a round-0 key
  kCtrIndexAux = kMaxPasses + 7,     // index builds: the row of $ in the transform
  kCtrPairI = kMaxPasses + 8,        // sort-based pairing: non-unique items paired this round
  kCtrPairU = kMaxPasses + 9,        // sort-based pairing: unique items kept for the next round
  kCtrStage = kMaxPasses + 10,       // staged ISA writes of the last re-rank
  kCtrCount = kMaxPasses + 11,
};

}  // namespace sa
