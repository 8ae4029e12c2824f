/*
 * sa.h -- C ABI of the MI355X (gfx950) suffix-array library.
 *
 * The library builds suffix arrays by prefix doubling with discarding
 * (Bingmann, Gog, Kurpicz, "Scalable Construction of Text Indexes",
 * arXiv 1610.03007, Section 2.1, Alg. 5 and 6, with the inverse-suffix-array
 * pairing of Alg. 4) entirely on one GPU with hand-written HIP kernels.
 *
 * Problem statement (Section 2): for a text T of length n over an alphabet,
 * suffix i is T[i, n); the suffix array SA is the permutation of [0, n) that
 * lists the suffixes in lexicographic order, and the inverse suffix array ISA
 * is its inverse. Here characters are bytes compared as unsigned values, and a
 * proper prefix is smaller than every extension of it (the end of the text
 * acts as a sentinel below every byte). The result is unique and bit-exact.
 *
 * Conventions for every entry point:
 *   - All functions return sa_status; nothing throws across the ABI.
 *   - Pointers named d_* are device pointers (hipMalloc or a PyTorch CUDA
 *     tensor) on the context's device; h_* are host pointers. The caller owns
 *     every buffer it passes; the context owns its workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *     is enqueued on it; the call returns after the result is complete on that
 *     stream (the call synchronizes with the stream once per doubling round).
 *   - On an error, outputs are undefined and the context stays usable.
 *   - A context must be used by one host thread at a time.
 */
#ifndef SA_MI355X_H
#define SA_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SA_OK = 0,
  SA_EINVAL = 1,   /* null pointer, bad size or flag, sigma outside [1, 256] */
  SA_ENOMEM = 2,   /* a workspace allocation failed */
  SA_ETOOBIG = 3,  /* n >= 2^32 (ranks and SA entries are 32-bit), or above an entry
                      point's stated maximum */
  SA_EDEVICE = 4,  /* a HIP call failed or a kernel reported an error */
  SA_EBUSY = 5     /* the resource is in use */
} sa_status;

typedef struct sa_ctx sa_ctx;

/* Creates a context on HIP device `device`. The workspace grows on demand and
 * is kept for later calls. tune_cache_json: optional path of a tuning cache
 * (may be NULL). The file is read once here; a missing file is an empty cache,
 * a malformed one gives SA_EINVAL. Builds without an explicit tuning take
 * their knobs from the cache entry that matches the input (see sa_tune). */
sa_status sa_ctx_create(sa_ctx** out, int device, const char* tune_cache_json);

/* Frees the context and its device workspace. NULL is accepted. */
sa_status sa_ctx_destroy(sa_ctx* ctx);

/* Suffix array of one text (Section 2 problem statement; method of Section
 * 2.1, Alg. 5).
 *   d_text: device u8[n], the text.
 *   n:      text length; n = 0 is a no-op; n >= 2^32 gives SA_ETOOBIG.
 *   sigma:  alphabet-size hint in [1, 256]; the result never depends on it
 *           (the library measures the alphabet itself).
 *   d_sa:   device u32[n], receives the suffix array (may be read through an
 *           int32 view; every value is < n).
 * Needs about 37 bytes of device workspace per text byte. */
sa_status sa_build(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma,
                   uint32_t* d_sa, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): sa_build
 * with no allocation of any kind. The workspace is a fixed device array built
 * into the library, SA_NOALLOC_MAX_N suffixes in size (about 40 MB; every GPU
 * the library runs on holds its own copy until the process ends), instead of
 * the context's workspace; the context supplies its tuning and its pinned
 * readback buffers, allocated when it was created. Arguments and result as
 * sa_build. n above SA_NOALLOC_MAX_N gives SA_ETOOBIG before anything is
 * enqueued. Every call on one GPU shares that GPU's array, whichever context
 * makes it: calls that overlap on one GPU (from several host threads or
 * several streams) race and must be serialised by the caller. Kernel tracing
 * is off for the call. */
#define SA_NOALLOC_MAX_N (1u << 20)
sa_status sa_build_noalloc(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma,
                           uint32_t* d_sa, void* stream);

/* Suffix arrays of many texts in one batched build: every doubling round runs
 * one sort and one re-rank launch for all texts together (the text id sits in
 * the high key bits), instead of one build per text.
 *   d_texts:   device u8[offsets[num_texts]], the texts concatenated.
 *   h_offsets: host u64[num_texts + 1], offsets[0] = 0, non-decreasing; text t is
 *              d_texts[offsets[t], offsets[t+1]) (empty texts are allowed).
 *   d_sas:     device u32[offsets[num_texts]]; text t's suffix array (local
 *              positions, values < n_t) is written to d_sas[offsets[t] ..).
 * Errors: SA_EINVAL for null pointers, num_texts = 0, offsets[0] != 0 or
 * decreasing offsets; SA_ETOOBIG if a text has 2^32 or more bytes, if
 * bits(num_texts - 1) + 2 * bits(longest text) > 64 (the key layout), or if
 * the total reaches 2^40 bytes. The total may exceed 2^32. Workspace: about 45
 * bytes per byte of all texts. */
sa_status sa_build_batch(sa_ctx* ctx, const uint8_t* d_texts, const uint64_t* h_offsets,
                         uint32_t num_texts, uint32_t* d_sas, void* stream);

/* Continuous-batching server. A worker thread owns the device work: requests
 * are admitted in arrival order while a slot is free and their text fits in
 * the server's device arena (their HBM footprint), and every loop runs one
 * merged doubling round for all admitted requests: new ones start round 0 while
 * the others do their own next round, in the same sort and re-rank launches.
 * A request's rank arrays stay on the device between rounds. Results equal
 * sa_build of the same text alone. */
typedef struct sa_server sa_server;
/* capacity_bytes: device memory the server may use (0 = half of the free
 * memory); max_text: longest accepted text (0 = 2^26). When max_text exceeds
 * 16 MiB the server runs two lanes on separate streams: texts up to 1 MiB
 * (a quarter of the memory) and longer texts, so short requests never wait
 * behind a long text's round. Each lane holds at most
 * 2^(64 - 2 * bits(lane max text)) requests (capped at 1024) in flight. */
sa_status sa_server_create(sa_server** out, int device, uint64_t capacity_bytes,
                           uint64_t max_text);
/* Stops the worker (requests still queued or running are dropped). */
sa_status sa_server_destroy(sa_server* srv);
/* Queues a copy of host text h_text[0, n); *ticket identifies the request.
 * The copy goes into a pinned host pool of the lane (up to 4 GiB) when it has
 * room, else into pageable memory. SA_ETOOBIG if n exceeds max_text or the
 * arena. */
sa_status sa_server_submit(sa_server* srv, const uint8_t* h_text, uint64_t n, uint64_t* ticket);
/* *done = 1 once the request finished: its suffix array is copied to
 * h_sa_out[0, n) and the request is released. h_sa_out may be host memory
 * (pinned memory gets one direct copy) or device memory of the server's GPU.
 * latency_ms (may be NULL) receives the time from submit to the suffix array
 * being complete on the device. *done = 0 while it is queued or running. With h_sa_out NULL a
 * finished request reports *done = 2 and stays until polled with a buffer.
 * A failed request returns its error once and is released; an unknown ticket
 * gives SA_EINVAL. */
sa_status sa_server_poll(sa_server* srv, uint64_t ticket, uint32_t* h_sa_out, int* done,
                         double* latency_ms);
typedef struct {
  uint64_t completed, failed, suffixes, rounds;
  double busy_ms;                    /* worker time spent in rounds */
  uint64_t queued, running, slots, arena_positions;
} sa_server_stats_t;
sa_status sa_server_stats(sa_server* srv, sa_server_stats_t* out);

/* Per-build diagnostics of the last sa_build / sa_build_batch / sa_build_rounds call. */
#define SA_MAX_ROUNDS 64
typedef struct {
  uint64_t n;
  uint32_t rounds;        /* doubling rounds run, round 0 included */
  uint32_t sigma;         /* distinct byte values in the text */
  uint32_t code_bits;     /* bits per character in a round-0 key */
  uint32_t chars0;        /* characters per round-0 key: the first prefix length */
  uint64_t prefix_len;    /* prefix length the ranks resolve after the last round */
  uint32_t lazy_isa;      /* 1 if the ISA was resolved lazily after round 0 */
  uint32_t graph_rounds;  /* enqueued later rounds replayed from a captured HIP graph
                             (sa_build / sa_build_rounds) */
  uint64_t dense_rounds;  /* bit k: round k was dense (most suffixes still active, so it
                             sorted all n with the names read in position order) */
  uint64_t active[SA_MAX_ROUNDS];       /* suffixes sorted in round k */
  uint32_t passes_run[SA_MAX_ROUNDS];   /* radix passes executed in round k */
  uint32_t key_bits[SA_MAX_ROUNDS];     /* key bits sorted in round k */
} sa_build_info;

sa_status sa_last_build_info(const sa_ctx* ctx, sa_build_info* out);

/* Runs at most `max_rounds` doubling rounds (0 = until done) and exposes the
 * intermediate state, for checking the method round by round.
 *   d_sa:  device u32[n]; positions finalised so far hold their suffix.
 *   d_isa: device u32[n] (may be NULL); receives the names after the last round
 *          run: ISA[i] = 1 + the number of suffixes whose prefix of length
 *          info.prefix_len is smaller than that of suffix i (Section 2.1,
 *          lexicographic names, here 1-based with 0 kept for the sentinel).
 * Other arguments as sa_build. Results are in sa_last_build_info. */
sa_status sa_build_rounds(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t max_rounds,
                          uint32_t* d_sa, uint32_t* d_isa, void* stream);

/* Prefix doubling with discarding by sorting (Section 2.1, Alg. 5 with the
 * comparator of Eq. 1 and the Unique / NPairs / renaming functions of Alg. 6):
 * the same suffix array as sa_build, built without an inverse suffix array.
 * Each round sorts the working items by (i mod h, i div h) so that suffix
 * i + h follows suffix i, pairs neighbours in one scan, keeps a unique item
 * only while the two items before it are non-unique (its name may still be
 * needed), sorts the non-unique items by name pair and renames them. This is
 * the form for a text sharded across devices, where ISA[i + h] is remote; on
 * one device it moves more bytes than sa_build.
 *   h_counts: host u64[4 * max_rounds] or NULL: for round k = 1, 2, ... the
 *             items sorted |P|, the non-unique items paired |I|, the items
 *             discarded (final) and the unique items kept.
 * Other arguments, errors and limits as sa_build; rounds and passes in
 * sa_last_build_info (active[k] = |P| of round k). */
sa_status sa_build_sorted_pairs(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma,
                                uint32_t* d_sa, uint64_t* h_counts, uint32_t max_rounds,
                                void* stream);

/* Suffix array by the difference cover algorithm DC3 (Section 2.2, Alg. 7): a
 * second suffix sorter, recursive on the suffixes at positions i mod 3 != 0.
 * Each level sorts their character triples and names them; equal names send
 * the names (positions 1, 4, 7, ... then 2, 5, 8, ...) to the next level,
 * whose suffix array orders them; the suffixes at i mod 3 == 0 are sorted by
 * (T[i], rank of i + 1), and the two lists are merged with the method's
 * comparison. Same result as sa_build.
 *   d_text, n, d_sa, stream: as sa_build (n < 2^32).
 *   d_rank12: device u32[n] or NULL: the top level's sample ranks, for each
 *             position i with i mod 3 != 0 the 1-based rank of suffix i among
 *             those suffixes, 0 where i mod 3 == 0.
 * Levels in sa_last_build_info: rounds = recursion levels, active[k] = the
 * length of the string at level k. Each level allocates its arrays (about
 * 4 bytes per symbol each) on top of the context's workspace. */
sa_status sa_build_dc3(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t* d_sa,
                       uint32_t* d_rank12, void* stream);

/* Suffix array by the difference cover algorithm DC7 (Section 2.2): the
 * sample is the suffixes at positions i mod 7 in {0, 1, 3}; their seven-
 * character tuples are sorted and named, equal names send the name string
 * (positions 0, 7, ... then 1, 8, ... then 3, 10, ...) to DC3, the other
 * four classes are sorted by (characters up to the next sample position, its
 * rank), and the five sorted lists are merged with the method's comparison
 * (at most six characters, then two sample ranks). Same result as sa_build.
 *   d_rank_sample: device u32[n] or NULL: for each position i with i mod 7 in
 *                  {0, 1, 3}, the 1-based rank of suffix i among those
 *                  suffixes; 0 at the other positions.
 * Levels in sa_last_build_info (rounds, active[k]); allocates its arrays
 * (about 70 bytes per text byte) on top of the context's workspace. */
sa_status sa_build_dc7(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t* d_sa,
                       uint32_t* d_rank_sample, void* stream);

/* The sorting step on its own (the Sort of Alg. 1 and 5): stable LSD radix
 * sort of `count` (key, value) pairs in place, ordered by the low `key_bits`
 * bits of the key (1..64; higher bits must be zero). d_keys: device u64[count],
 * d_vals: device u32[count]. */
sa_status sa_radix_sort_pairs(sa_ctx* ctx, uint64_t* d_keys, uint32_t* d_vals, uint64_t count,
                              uint32_t key_bits, void* stream);

/* How the inverse suffix array is formed after round 0 (a tuning choice; the
 * result is the same). Eager: one random 4-byte write per suffix. Lazy: only
 * the suffixes that survive round 0 are written, and a later round that needs
 * the round-0 name of another suffix recomputes it by binary search in the
 * round-0 sorted keys. Auto picks lazy when at most 1/lazy_ratio of the
 * suffixes survive (sa_tuning; 8 by default). Lazy needs the survivors to fit
 * in spare workspace (at most n/3); otherwise eager is used. The mode applies
 * to sa_build, sa_build_rounds and sa_build_batch (n: all texts' suffixes);
 * the server always forms the ISA eagerly, since its texts join at any round. */
enum { SA_ISA_AUTO = 0, SA_ISA_EAGER = 1, SA_ISA_LAZY = 2 };
sa_status sa_ctx_set_isa_mode(sa_ctx* ctx, int mode);

/* Tuning knobs (none changes a result). Unknown or unsupported values give
 * SA_EINVAL and leave the context unchanged. Defaults: 512-thread sweep
 * workgroups of 8 items, the workgroups one CU holds, lazy_ratio 8, trimmed
 * round-0 keys. */
typedef struct {
  uint32_t sort_items;   /* radix-sort items per thread: 8, 12, 16, 20 or 24 with 256-thread
                            workgroups (tile = sort_block x sort_items) */
  uint32_t lazy_ratio;   /* auto ISA mode is lazy when survivors <= n / lazy_ratio (>= 3) */
  uint32_t round0_full;  /* 1: pack floor(64 / code bits) characters in round 0; 0 (default):
                            drop the characters that only half-fill a last 8-bit digit */
  uint32_t sort_wgs_per_cu; /* persistent radix-sweep workgroups per compute unit
                               (0 = what one CU holds for the tile shape; at most 16) */
  uint32_t sort_block;   /* radix-sweep workgroup size: 256 (0 means 256) or 512; with 512,
                            sort_items is 4, 8 or 12 */
  uint32_t sort_match;   /* how a sweep wave finds the lanes that hold the same digit:
                            0 (default) = eight ballots, whose cost does not depend on the
                            digits; 1 = an LDS table (fewer instructions, but lanes of
                            equal digits collide in its atomics) */
  uint32_t radix_bits;   /* radix-sort digit width in bits: 0 (default) = 8 */
  uint32_t rounds_ahead; /* doubling rounds after round 0 enqueued before the host reads the
                            survivor count back: 0 (default) = 1, then 2, 4, ... up to 16
                            per readback; k in [1, 64] = k each time. A round that finds no
                            survivor does nothing. */
  uint32_t round_graphs; /* 0 (default): a later round whose launch arguments repeat is
                            captured once as a HIP graph and replayed; 1: every kernel is
                            launched directly. Tracing always launches directly. */
  uint32_t prefix_mult;  /* names resolve prefix lengths multiplied per later round by: 0 or 2
                            (default) = prefix doubling, rank pairs; 4 = prefix quadrupling
                            (Section 2.1): rank quadruples sorted as two 2b-bit words, half
                            the rounds, always with the eager ISA. sa_build and
                            sa_build_rounds only; batches and the server double. */
  uint32_t isa_direct;   /* 0 (default): in a single text of at least 2^26 bytes, a round with
                            at least 2^22 active suffixes writes its names into the ISA grouped
                            by position (256 buckets, one after the other); 1: every name is
                            written straight from the re-rank. */
} sa_tuning;
/* Sets an explicit tuning, used by every later build of the context. t = NULL
 * goes back to automatic choice: the cache entry for each input, else the
 * defaults. */
sa_status sa_ctx_set_tuning(sa_ctx* ctx, const sa_tuning* t);
/* The knobs of the last build (or the explicit tuning, or the defaults). */
sa_status sa_ctx_get_tuning(const sa_ctx* ctx, sa_tuning* out);
/* Where the last build's knobs came from: 0 defaults, 1 the tuning cache,
 * 2 an explicit sa_ctx_set_tuning. */
sa_status sa_ctx_tuning_source(const sa_ctx* ctx, int* source);

/* Autotuner. Times candidate tunings on the caller's input and records the
 * fastest in the context's cache table, keyed by (GPU architecture, mode,
 * floor(log2 of the total length), bits per character code of the input):
 *   stage 1: (sort_items, sort_block) in {8, 12, 16, 20, 24} x 256 and
 *            {4, 8, 12} x 512, x sort_wgs_per_cu in {default, 1, 2, 3, 4};
 *   stage 2: sort_match 1 (the LDS table);
 *   stage 3: round0_full flipped; stage 4: lazy_ratio in {3, 4, 8, 16, 64}.
 * Each candidate is one warm-up build plus the best of `reps` timed builds
 * (0 = 3) on `stream`, measured with HIP events. d_texts / h_offsets /
 * num_texts / d_sas are as sa_build_batch (num_texts = 1 tunes sa_build,
 * mode "single"; more tunes the batched build, mode "batch"). d_sas receives
 * a valid result. *best_out (may be NULL) gets the winner, *best_ms (may be
 * NULL) its time. The caller's explicit tuning, if any, stays in force.
 * A later build finds the entry when it has the same architecture and mode, a
 * size within two binary orders of magnitude (nearest first) and, for
 * sa_build, the nearest code width to bits(sigma hint) (a hint of 256 matches
 * any width). With SA_TUNE_LOG set in the environment, each candidate's time
 * is printed to stderr. */
sa_status sa_tune(sa_ctx* ctx, const uint8_t* d_texts, const uint64_t* h_offsets,
                  uint32_t num_texts, uint32_t* d_sas, void* stream, uint32_t reps,
                  sa_tuning* best_out, double* best_ms);
/* Writes the context's cache table as JSON to `path` (NULL: the path given to
 * sa_ctx_create). The file is replaced atomically. */
sa_status sa_tune_save(const sa_ctx* ctx, const char* path);
/* Host-only lookup in a cache file (no device needed): the tuning a build of
 * n bytes in `mode` ("single" or "batch") on `arch` (e.g. "gfx950") with
 * code_bits bits per character (0: any) would take; *found = 0 and the
 * defaults when no entry matches. A missing file is an empty cache. */
sa_status sa_tune_lookup(const char* path, const char* arch, const char* mode, uint64_t n,
                         uint32_t code_bits, sa_tuning* out, int* found);

/* ---------------------------------------------------------------------------
 * Index structures from a text and its suffix array, on the device. The
 * paper's conclusion names these as the next step after suffix sorting: the
 * LCP array and further text indexes built from the suffix array. d_sa must be
 * the suffix array of d_text (as sa_build writes it); an array that is not a
 * permutation of [0, n) gives SA_EDEVICE or undefined outputs, never a fault.
 * Each call returns when its result is complete on `stream`. */

/* LCP array: d_lcp[0] = 0 and, for j >= 1, d_lcp[j] = the number of leading
 * bytes suffixes d_sa[j - 1] and d_sa[j] have in common. d_lcp: device u32[n].
 * Uses 4n + n/8 bytes of the context's workspace (which grows to a build's
 * size). Method: each entry compared directly over at most 32 bytes; the
 * entries that reach 32 follow from Kasai et al.'s bound
 * lcp(i + 1) >= lcp(i) - 1 along the text, in the permuted (Phi) form. Every
 * step runs in the library's kernels. */
sa_status sa_lcp(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, const uint32_t* d_sa,
                 uint32_t* d_lcp, void* stream);

/* Burrows-Wheeler transform of text$, $ below every byte: the rows are the
 * suffixes of text$ in sorted order ($ alone first, then d_sa[0], d_sa[1],
 * ...), and the transform lists the character before each row (cyclically:
 * text[n - 1] before $ alone, $ before the whole text). d_bwt: device u8[n]
 * receives it with its single $ left out; *dollar (host) the row of the $,
 * in [1, n] (0 when n = 0). */
sa_status sa_bwt(sa_ctx* ctx, const uint8_t* d_text, uint64_t n, const uint32_t* d_sa,
                 uint8_t* d_bwt, uint64_t* dollar, void* stream);

/* FM index of a text: its transform and occurrence counts sampled every 256
 * rows for each byte present, in device memory the index owns (about
 * n + 4 n sigma / 256 bytes). Built from the text and its suffix array; the
 * caller's buffers are not kept. */
typedef struct sa_fm sa_fm;
sa_status sa_fm_create(sa_fm** out, sa_ctx* ctx, const uint8_t* d_text, uint64_t n,
                       const uint32_t* d_sa, void* stream);
/* Pattern queries by backward search, one pattern per wavefront.
 *   d_patterns:  device u8, the patterns concatenated (may be NULL if all are
 *                empty);
 *   d_offsets:   device u64[num_patterns + 1]: pattern q is
 *                d_patterns[d_offsets[q], d_offsets[q + 1]);
 *   d_ranges:    device u64[2 num_patterns]: for pattern q, [lo, hi) = the
 *                positions of the suffix array whose suffixes start with it
 *                (hi - lo occurrences; when there are none, lo = hi = the number
 *                of suffixes smaller than the pattern). The empty pattern gives
 *                [0, n).
 * Enqueued on `stream` without waiting. */
sa_status sa_fm_count(sa_fm* fm, const uint8_t* d_patterns, const uint64_t* d_offsets,
                      uint32_t num_patterns, uint64_t* d_ranges, void* stream);
/* Text length, row of $, bytes present and device bytes of an index (any
 * output pointer may be NULL). */
sa_status sa_fm_info(const sa_fm* fm, uint64_t* n, uint64_t* dollar, uint32_t* sigma,
                     uint64_t* device_bytes);
sa_status sa_fm_destroy(sa_fm* fm);

/* Device workspace (bytes) a context needs to build `num_texts` texts of
 * `total_n` bytes in all: sa_build when num_texts <= 1 (about 37 bytes per text
 * byte), sa_build_batch otherwise (about 45 bytes per byte of all texts, plus
 * a table row of about 600 bytes per text). Host-only; for admission and
 * planning. The caller's text and SA buffers are not included. */
size_t sa_workspace_bytes(uint64_t total_n, uint32_t num_texts);

/* Per-kernel timing. With tracing on, every kernel launch of a build is
 * bracketed by HIP events on the build's stream; the totals accumulate until
 * reset. `kind` selects the kernel (SA_KERNEL_*). bytes are the algorithmic
 * bytes of those launches (what the step must read and write, random 4-byte
 * accesses counted at 4 bytes). */
enum {
  SA_KERNEL_SORT_PASS = 0,   /* one radix-sort sweep */
  SA_KERNEL_HISTOGRAM = 1,   /* up-front digit histograms */
  SA_KERNEL_RERANK = 2,      /* re-rank, ISA scatter, finalise, compact */
  SA_KERNEL_PACK_TEXT = 3,   /* round-0 keys from the text */
  SA_KERNEL_PACK_PAIRS = 4,  /* round >= 1 keys (ISA gather) */
  SA_KERNEL_OTHER = 5,       /* alphabet, plan, fills */
  SA_KERNEL_ISA_SCATTER = 6, /* eager ISA after round 0 */
  SA_KERNEL_KINDS = 7
};
typedef struct {
  uint64_t launches;
  double ms;
  double bytes;
} sa_kernel_stats;

sa_status sa_ctx_set_trace(sa_ctx* ctx, int on);
sa_status sa_ctx_reset_stats(sa_ctx* ctx);
sa_status sa_ctx_get_kernel_stats(const sa_ctx* ctx, int kind, sa_kernel_stats* out);

const char* sa_strerror(sa_status s);

#ifdef __cplusplus
}
#endif

#endif /* SA_MI355X_H */
