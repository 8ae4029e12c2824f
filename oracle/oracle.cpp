// Oracle for suffix-array construction by prefix doubling.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or load
// this file; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark do. It shares no code, header, table or helper with the HIP library.
//
// Everything here is plain, single-pass-per-step C++17 on the host. Sorting is
// std::sort (built with -D_GLIBCXX_PARALLEL it becomes the GNU parallel sort,
// which is how the multi-core CPU baseline is produced; the arithmetic is the
// same). Ranks and indices are uint32_t, so n < 2^32.
//
// Conventions (paper, Section 2, problem statement and Section 2.1):
//  * A suffix i is T[i, n). Bytes compare as unsigned 8-bit values, and a proper
//    prefix is smaller than any extension of it: the past-the-end sentinel `$`
//    is smaller than every byte, including 0x00.
//  * Names are 1-based head ranks: the name of a suffix for prefix length h is
//    1 + the number of suffixes whose length-h prefix is strictly smaller. The
//    value 0 is reserved for the sentinel `$` (the paper's worked examples give
//    the smallest group the name 0 while also using 0 as the sentinel name; the
//    two would collide, so every name here is the paper's name + 1).
//
// Parity status: every function below is pinned by tests that do not call it
// to produce their expected values (paper worked examples, brute force written
// independently in Python, closed forms, and planted-mistake mutants).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <utility>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// One item of the paper's triple array S: a text position and its name pair.
struct Triple {
  uint64_t pair;  // (r0 << 32) | r1 ; r1 == 0 is the sentinel
  uint32_t i;
};

// Sort S by name pair, then give every item the name 1 + (position of the last
// item whose name pair differs from its predecessor). This is the paper's
// name-comparison function (Alg. 2) followed by the max-PrefixSum of Alg. 1,
// shifted to 1-based names. Returns the number of distinct name pairs.
uint64_t sort_and_name(std::vector<Triple>& S, uint32_t* name) {
  std::sort(S.begin(), S.end(),
            [](const Triple& a, const Triple& b) { return a.pair < b.pair; });
  uint64_t last_head = 0, distinct = 0;
  for (uint64_t p = 0; p < S.size(); ++p) {
    if (p == 0 || S[p].pair != S[p - 1].pair) {
      last_head = p;
      ++distinct;
    }
    name[S[p].i] = static_cast<uint32_t>(last_head + 1);
  }
  return distinct;
}

// Prefix doubling (Alg. 1) with the pairing of Alg. 4: the name of suffix i+h is
// read from the partial inverse suffix array (the name array indexed by text
// position), or is the sentinel 0 when i+h >= n.
// Runs at most `max_steps` sorts (0 = until every name is distinct) and leaves
// the names in `name`; *h_out receives the prefix length those names resolve.
void prefix_doubling(const uint8_t* T, uint64_t n, uint64_t max_steps,
                     uint32_t* name, uint64_t* h_out) {
  std::vector<Triple> S(n);
  // Initial triples (i, T[i], T[i+1]) with T[n] = `$`. Characters are shifted by
  // one so that 0 stays the sentinel.
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t c0 = uint64_t(T[i]) + 1;
    uint64_t c1 = (i + 1 < n) ? uint64_t(T[i + 1]) + 1 : 0;
    S[i] = Triple{(c0 << 32) | c1, static_cast<uint32_t>(i)};
  }
  uint64_t h = 2;  // prefix length resolved by the names after the next sort
  uint64_t steps = 0;
  for (;;) {
    uint64_t distinct = sort_and_name(S, name);
    ++steps;
    if (distinct == n) break;                       // every name is unique
    if (max_steps != 0 && steps >= max_steps) break;
    // Next name pairs: own name and the name h positions to the right.
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t r0 = name[i];
      uint64_t r1 = (i + h < n) ? name[i + h] : 0;
      S[i] = Triple{(r0 << 32) | r1, static_cast<uint32_t>(i)};
    }
    h *= 2;
  }
  if (h_out) *h_out = h;
}

// Padded-prefix comparison: T[i, min(i+h, n)) versus T[j, min(j+h, n)), unsigned
// bytes, a proper prefix being the smaller. Returns <0, 0, >0.
int cmp_prefix(const uint8_t* T, uint64_t n, uint64_t h, uint64_t i, uint64_t j) {
  uint64_t li = std::min<uint64_t>(h, n - i);
  uint64_t lj = std::min<uint64_t>(h, n - j);
  uint64_t l = std::min(li, lj);
  int c = (l > 0) ? std::memcmp(T + i, T + j, l) : 0;
  if (c != 0) return c;
  if (li == lj) return 0;
  return li < lj ? -1 : 1;
}

}  // namespace

extern "C" {

// Suffix array of T[0, n) by plain prefix doubling (no discarding): every
// suffix is re-sorted every round until all names are distinct; then
// SA[name[i] - 1] = i. Returns 0, or 1 if n >= 2^32.
int oracle_sa(const uint8_t* T, uint64_t n, uint32_t* SA) {
  if (n >= (uint64_t(1) << 32)) return 1;
  if (n == 0) return 0;
  if (n == 1) {
    SA[0] = 0;
    return 0;
  }
  std::vector<uint32_t> name(n);
  prefix_doubling(T, n, 0, name.data(), nullptr);
  for (uint64_t i = 0; i < n; ++i) SA[name[i] - 1] = static_cast<uint32_t>(i);
  return 0;
}

// Names after `steps` doubling sorts (steps >= 1; the first sort resolves
// prefix length 2, each further one doubles it), or after the sort that makes
// every name distinct if that comes first. *h_out = prefix length resolved.
int oracle_pd_names(const uint8_t* T, uint64_t n, uint64_t steps, uint32_t* names,
                    uint64_t* h_out) {
  if (n >= (uint64_t(1) << 32) || steps == 0) return 1;
  if (n == 0) {
    *h_out = 0;
    return 0;
  }
  if (n == 1) {
    names[0] = 1;
    *h_out = 2;
    return 0;
  }
  prefix_doubling(T, n, steps, names, h_out);
  return 0;
}

// Prefix a-tupling (Section 2.1, "Prefix Quadrupling": a = 4; a = 2 is plain
// doubling): the names start from single characters (prefix length 1), and each
// sort orders the a-tuples (name[i], name[i+h], ..., name[i+(a-1)h]) with the
// sentinel 0 past the end, renames them as in Alg. 2 and the max-PrefixSum,
// and multiplies the resolved prefix length h by a. Runs at most `steps` tuple
// sorts (no sort at all for 0: the names of single characters), stopping early
// once every name is distinct, and leaves the names in `name`; *h_out = the
// prefix length they resolve. Returns 0, or 1 for n >= 2^32 or a < 2.
int oracle_pa_names(const uint8_t* T, uint64_t n, uint32_t a, uint64_t steps, uint32_t* name,
                    uint64_t* h_out) {
  if (n >= (uint64_t(1) << 32) || a < 2) return 1;
  *h_out = 1;
  if (n == 0) return 0;
  // Names of single characters: 1 + the number of positions holding a smaller byte.
  uint64_t below[257] = {0};
  for (uint64_t i = 0; i < n; ++i) below[uint64_t(T[i]) + 1] += 1;
  for (int c = 1; c <= 256; ++c) below[c] += below[c - 1];
  uint64_t distinct = 0;
  for (int c = 0; c < 256; ++c) distinct += below[c + 1] != below[c];
  for (uint64_t i = 0; i < n; ++i) name[i] = static_cast<uint32_t>(below[T[i]] + 1);
  uint64_t h = 1, done = 0;
  std::vector<uint32_t> tup(n * uint64_t(a));
  std::vector<uint32_t> idx(n);
  while (distinct < n && done < steps) {
    for (uint64_t i = 0; i < n; ++i)
      for (uint32_t j = 0; j < a; ++j) {
        const uint64_t q = i + uint64_t(j) * h;
        tup[i * a + j] = q < n ? name[q] : 0;
      }
    std::iota(idx.begin(), idx.end(), 0u);
    auto less = [&](uint32_t x, uint32_t y) {
      return std::lexicographical_compare(&tup[uint64_t(x) * a], &tup[uint64_t(x) * a] + a,
                                          &tup[uint64_t(y) * a], &tup[uint64_t(y) * a] + a);
    };
    auto same = [&](uint32_t x, uint32_t y) {
      return std::equal(&tup[uint64_t(x) * a], &tup[uint64_t(x) * a] + a,
                        &tup[uint64_t(y) * a]);
    };
    std::sort(idx.begin(), idx.end(), less);
    uint64_t head = 0;
    distinct = 0;
    for (uint64_t p = 0; p < n; ++p) {
      if (p == 0 || !same(idx[p - 1], idx[p])) {
        head = p;
        ++distinct;
      }
      name[idx[p]] = static_cast<uint32_t>(head + 1);
    }
    h *= a;
    ++done;
  }
  *h_out = h;
  return 0;
}

// Suffix array by prefix a-tupling: names until all are distinct, then
// SA[name[i] - 1] = i.
int oracle_pa_sa(const uint8_t* T, uint64_t n, uint32_t a, uint32_t* SA) {
  if (n >= (uint64_t(1) << 32) || a < 2) return 1;
  std::vector<uint32_t> name(n);
  uint64_t h = 0;
  oracle_pa_names(T, n, a, ~uint64_t(0), name.data(), &h);
  for (uint64_t i = 0; i < n; ++i) SA[name[i] - 1] = static_cast<uint32_t>(i);
  return 0;
}

// ---------------------------------------------------------------------------
// Prefix doubling with discarding by sorting (Alg. 5 with the comparator of
// Eq. 1 and the helper functions of Alg. 6): no inverse suffix array; each
// round sorts the working items by text position in the comparator's order so
// that suffix i and suffix i + h are neighbours, pairs them in one scan, and
// keeps a unique item only while a non-unique item may still need its name.
// Readings: names are 1-based (0 is the sentinel); the window arrays' length
// l is the number of items; the last window is the one ending at the last
// item; the non-unique items are sorted by name pair before renaming; a new
// name is the old one plus the offset of the item's run of equal pairs inside
// its group of equal old names; the loop ends when no item is non-unique.

// Positions 0..n-1 in the order of Eq. 1 for offset h: by i mod h, then by
// i div h (h = 2^k in the paper; any h >= 1 here).
int oracle_opk_order(uint64_t n, uint64_t h, uint32_t* out) {
  if (n >= (uint64_t(1) << 32) || h == 0) return 1;
  std::vector<uint32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0u);
  std::sort(idx.begin(), idx.end(), [h](uint32_t a, uint32_t b) {
    if (a % h != b % h) return a % h < b % h;
    return a / h < b / h;
  });
  std::copy(idx.begin(), idx.end(), out);
  return 0;
}

namespace {

struct Item {
  uint32_t i, r;
  char s;  // 'u' unique, 'n' not unique
};

// Alg. 5 from names of c-character prefixes. Runs until no item is
// non-unique, or stops before round max_rounds + 1 (0: no limit). Per round k
// (1-based) appends |P|, |I|, |D'|, |U'| to `counts` and, when k == snap_round,
// copies P (sorted by the comparator, with the states) to snap.
uint64_t sort_discarding(const uint8_t* T, uint64_t n, uint64_t c, uint32_t* SA,
                         std::vector<uint64_t>* counts, uint64_t max_rounds,
                         uint64_t snap_round, std::vector<Item>* snap) {
  // Initial names: 1 + the number of suffixes whose c-prefix is smaller, with
  // the items in name order (the sorted triples of the initial step, which
  // uses c = 2).
  std::vector<uint32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0u);
  std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
    return cmp_prefix(T, n, c, a, b) < 0;
  });
  std::vector<Item> N(n);
  uint64_t head = 0;
  for (uint64_t p = 0; p < n; ++p) {
    if (p > 0 && cmp_prefix(T, n, c, idx[p - 1], idx[p]) != 0) head = p;
    N[p] = Item{idx[p], static_cast<uint32_t>(head + 1), 'n'};
  }
  std::vector<Item> U;
  uint64_t h = c, round = 0;
  for (;;) {
    ++round;
    // Unique: in name order, an item is unique if its name differs from both
    // neighbours' (the first and last compare with their one neighbour).
    const uint64_t l = N.size();
    for (uint64_t j = 0; j < l; ++j) {
      const bool differs_prev = j == 0 || N[j - 1].r != N[j].r;
      const bool differs_next = j + 1 == l || N[j + 1].r != N[j].r;
      N[j].s = (differs_prev && differs_next) ? 'u' : 'n';
    }
    // Union with the kept unique items, sorted by the comparator of Eq. 1.
    std::vector<Item> P = N;
    P.insert(P.end(), U.begin(), U.end());
    std::sort(P.begin(), P.end(), [h](const Item& a, const Item& b) {
      if (a.i % h != b.i % h) return a.i % h < b.i % h;
      return a.i / h < b.i / h;
    });
    if (round == snap_round && snap) *snap = P;
    // NPairs over windows of three: a non-unique item takes the name of its
    // successor if that is suffix i + h (else the sentinel 0); a unique item is
    // kept only if the two items before it are both non-unique (one of them may
    // need its name in the next round), otherwise discarded: its name is final.
    std::vector<std::pair<uint64_t, uint32_t>> I;  // (r0 << 32 | r1, i)
    std::vector<Item> Unext;
    uint64_t discarded = 0;
    const uint64_t m = P.size();
    for (uint64_t p = 0; p < m; ++p) {
      const Item& x = P[p];
      if (x.s == 'n') {
        const bool next = p + 1 < m && uint64_t(P[p + 1].i) == uint64_t(x.i) + h;
        const uint64_t r1 = next ? P[p + 1].r : 0;
        I.push_back({(uint64_t(x.r) << 32) | r1, x.i});
      } else if (p >= 2 && P[p - 1].s == 'n' && P[p - 2].s == 'n') {
        Unext.push_back(x);
      } else {
        SA[x.r - 1] = x.i;
        ++discarded;
      }
    }
    if (counts) {
      counts->push_back(m);
      counts->push_back(I.size());
      counts->push_back(discarded);
      counts->push_back(Unext.size());
    }
    U = Unext;
    if (I.empty()) break;
    if (max_rounds != 0 && round >= max_rounds) break;
    // Sort the non-unique items by name pair and rename: old name + (start of
    // the run of equal pairs - start of the group of equal old names).
    std::sort(I.begin(), I.end());
    N.assign(I.size(), Item{0, 0, 'n'});
    uint64_t run = 0, grp = 0;
    for (uint64_t p = 0; p < I.size(); ++p) {
      if (p > 0 && I[p].first != I[p - 1].first) run = p;
      if (p > 0 && (I[p].first >> 32) != (I[p - 1].first >> 32)) grp = p;
      const uint64_t r0 = I[p].first >> 32;
      N[p] = Item{I[p].second, static_cast<uint32_t>(r0 + run - grp), 'n'};
    }
    h *= 2;
  }
  return round;
}

}  // namespace

// Suffix array by sort-based prefix doubling with discarding, from names of
// c-character prefixes (c = 2 is the paper's initial step). counts (may be
// NULL) receives |P|, |I|, |D'|, |U'| of every round, at most max_counts
// rounds; *rounds_out the number of rounds. Returns 0, or 1 on bad input.
int oracle_pdd_sa(const uint8_t* T, uint64_t n, uint64_t c, uint32_t* SA, uint64_t* counts,
                  uint64_t max_counts, uint64_t* rounds_out) {
  if (n >= (uint64_t(1) << 32) || c == 0) return 1;
  *rounds_out = 0;
  if (n == 0) return 0;
  std::vector<uint64_t> cnt;
  *rounds_out = sort_discarding(T, n, c, SA, &cnt, 0, 0, nullptr);
  if (counts)
    for (uint64_t k = 0; k < cnt.size() && k < 4 * max_counts; ++k) counts[k] = cnt[k];
  return 0;
}

// The working items P of round k (>= 1) after the comparator sort: positions,
// names and states ('u' = 1, 'n' = 0); *m receives |P| (the arrays hold n).
// Returns 1 if the build ended before round k.
int oracle_pdd_round(const uint8_t* T, uint64_t n, uint64_t c, uint64_t k, uint32_t* pos,
                     uint32_t* names, uint8_t* unique, uint64_t* m) {
  if (n >= (uint64_t(1) << 32) || c == 0 || k == 0) return 1;
  *m = 0;
  if (n == 0) return 1;
  std::vector<uint32_t> sa(n);
  std::vector<Item> P;
  const uint64_t rounds = sort_discarding(T, n, c, sa.data(), nullptr, k, k, &P);
  if (rounds < k) return 1;
  *m = P.size();
  for (uint64_t p = 0; p < P.size(); ++p) {
    pos[p] = P[p].i;
    names[p] = P[p].r;
    unique[p] = P[p].s == 'u' ? 1 : 0;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Difference cover DC3 (Section 2.2): the ranks of the sample suffixes, those
// starting at positions i with i mod 3 != 0, among themselves. r1[t] is the
// 1-based rank of suffix 3t + 1 (t < #{i < n : i mod 3 == 1}), r2[t] that of
// suffix 3t + 2. By definition: the sample positions in suffix-array order
// (the suffix array from the prefix-doubling function above).
int oracle_dc3_sample_ranks(const uint8_t* T, uint64_t n, uint32_t* r1, uint32_t* r2) {
  if (n >= (uint64_t(1) << 32)) return 1;
  if (n == 0) return 0;
  std::vector<uint32_t> sa(n);
  oracle_sa(T, n, sa.data());
  uint32_t rank = 0;
  for (uint64_t j = 0; j < n; ++j) {
    const uint64_t i = sa[j];
    if (i % 3 == 0) continue;
    ++rank;
    if (i % 3 == 1)
      r1[i / 3] = rank;
    else
      r2[i / 3] = rank;
  }
  return 0;
}

// Difference cover sample ranks for any cover (DC7: X = 7, D = {0, 1, 3};
// DC3: X = 3, D = {1, 2}): out[i] = 1-based rank of suffix i among the
// suffixes whose start i has i mod X in D, 0 for the others. `dmask` has bit
// d set for d in D. By definition, from the suffix array.
int oracle_dcx_sample_ranks(const uint8_t* T, uint64_t n, uint32_t X, uint32_t dmask,
                            uint32_t* out) {
  if (n >= (uint64_t(1) << 32) || X == 0 || X > 32) return 1;
  if (n == 0) return 0;
  std::vector<uint32_t> sa(n);
  oracle_sa(T, n, sa.data());
  uint32_t rank = 0;
  for (uint64_t i = 0; i < n; ++i) out[i] = 0;
  for (uint64_t j = 0; j < n; ++j) {
    const uint64_t i = sa[j];
    if ((dmask >> (i % X)) & 1u) out[i] = ++rank;
  }
  return 0;
}

// Closed form of the names for prefix length h: ranks[i] = 1 + #{ j :
// pad_h(j) < pad_h(i) }, where pad_h(i) is T[i, i+h) cut at n (the sentinel
// ending it). Computed by sorting positions with the padded-prefix comparison.
int oracle_prefix_ranks(const uint8_t* T, uint64_t n, uint64_t h, uint32_t* ranks) {
  if (n >= (uint64_t(1) << 32) || h == 0) return 1;
  std::vector<uint32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0u);
  std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
    return cmp_prefix(T, n, h, a, b) < 0;
  });
  uint64_t head = 0;
  for (uint64_t p = 0; p < n; ++p) {
    if (p > 0 && cmp_prefix(T, n, h, idx[p - 1], idx[p]) != 0) head = p;
    ranks[idx[p]] = static_cast<uint32_t>(head + 1);
  }
  return 0;
}

// Brute force from the definition: sort all suffix start positions with a
// lexicographic comparison of unsigned bytes (shorter prefix first).
int oracle_brute_sa(const uint8_t* T, uint64_t n, uint32_t* SA) {
  if (n >= (uint64_t(1) << 32)) return 1;
  std::vector<uint32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0u);
  std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
    return std::lexicographical_compare(T + a, T + n, T + b, T + n);
  });
  std::copy(idx.begin(), idx.end(), SA);
  return 0;
}

// Linear-time suffix array check (Burkhardt and Kaerkkaeinen, CPM 2003): SA is
// the suffix array of T iff it is a permutation of [0, n) and for every
// adjacent pair (a, b) = (SA[j], SA[j+1]):  T[a] < T[b], or T[a] == T[b] and
// R[a+1] < R[b+1], where R is the inverse of the SA under test (1-based) and
// R[n] = 0 stands for the empty suffix.
// Returns 0 if correct, 1 if not a permutation, 2 if an order violation;
// *where receives the offending position of SA.
int oracle_check_sa(const uint8_t* T, uint64_t n, const uint32_t* SA, uint64_t* where) {
  *where = 0;
  if (n >= (uint64_t(1) << 32)) return 1;
  std::vector<uint32_t> R(n + 1, 0);
  for (uint64_t j = 0; j < n; ++j) {
    uint64_t s = SA[j];
    if (s >= n || R[s] != 0) {
      *where = j;
      return 1;
    }
    R[s] = static_cast<uint32_t>(j + 1);
  }
  for (uint64_t j = 0; j + 1 < n; ++j) {
    uint64_t a = SA[j], b = SA[j + 1];
    bool ok = (T[a] < T[b]) || (T[a] == T[b] && R[a + 1] < R[b + 1]);
    if (!ok) {
      *where = j;
      return 2;
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Index structures derived from a suffix array. The paper's conclusion names
// the LCP array and further text indexes built from the suffix array as the
// next step; each function below is the plain definition of its output,
// computed from the text and a suffix array given by the caller.

// LCP array: lcp[0] = 0 and, for j >= 1, lcp[j] = the number of leading bytes
// suffixes SA[j - 1] and SA[j] have in common, counted byte by byte.
int oracle_lcp(const uint8_t* T, uint64_t n, const uint32_t* SA, uint32_t* lcp) {
  if (n == 0) return 0;
  lcp[0] = 0;
  for (uint64_t j = 1; j < n; ++j) {
    const uint64_t a = SA[j - 1], b = SA[j];
    if (a >= n || b >= n) return 1;
    uint64_t l = 0;
    while (a + l < n && b + l < n && T[a + l] == T[b + l]) ++l;
    lcp[j] = static_cast<uint32_t>(l);
  }
  return 0;
}

// Burrows-Wheeler transform of T$ ($ below every byte): the suffixes of T$ in
// sorted order are $ alone, then T[SA[0], n)$, T[SA[1], n)$, ...; the
// transform lists the character before each of them, read cyclically (T[n - 1]
// before $ alone, $ before the whole text). out[0, n) receives that column with
// its one $ left out, and *dollar the row where the $ stands.
int oracle_bwt(const uint8_t* T, uint64_t n, const uint32_t* SA, uint8_t* out, uint64_t* dollar) {
  *dollar = 0;
  if (n == 0) return 0;
  uint64_t k = 0;
  out[k++] = T[n - 1];
  for (uint64_t j = 0; j < n; ++j) {
    if (SA[j] >= n) return 1;
    if (SA[j] == 0) {
      *dollar = j + 1;
      continue;
    }
    out[k++] = T[SA[j] - 1];
  }
  return 0;
}

namespace {

// Compares the first m bytes of suffix s with P: negative if the suffix's
// prefix is smaller (a suffix that ends first is smaller), 0 if the suffix
// starts with P, positive if greater.
int cmp_prefix(const uint8_t* T, uint64_t n, uint64_t s, const uint8_t* P, uint64_t m) {
  for (uint64_t l = 0; l < m; ++l) {
    if (s + l >= n) return -1;
    if (T[s + l] != P[l]) return T[s + l] < P[l] ? -1 : 1;
  }
  return 0;
}

}  // namespace

// The positions [*lo, *hi) of the suffix array whose suffixes start with
// P[0, m) (contiguous, as the suffixes are sorted): two binary searches with
// byte comparisons. An empty pattern gives [0, n).
int oracle_sa_interval(const uint8_t* T, uint64_t n, const uint32_t* SA, const uint8_t* P,
                       uint64_t m, uint64_t* lo, uint64_t* hi) {
  uint64_t a = 0, b = n;
  while (a < b) {  // first j whose suffix is not below P
    const uint64_t mid = a + (b - a) / 2;
    if (cmp_prefix(T, n, SA[mid], P, m) < 0)
      a = mid + 1;
    else
      b = mid;
  }
  *lo = a;
  b = n;
  while (a < b) {  // first j whose suffix is above P
    const uint64_t mid = a + (b - a) / 2;
    if (cmp_prefix(T, n, SA[mid], P, m) <= 0)
      a = mid + 1;
    else
      b = mid;
  }
  *hi = a;
  return 0;
}

// Number of threads the parallel sort may use (1 in the sequential build).
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
