// FP64 CPU oracle for symmetric sparse kernels over the fully expanded tensor.
//
// TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
// definition that the GPU library is checked against. Only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it. It shares
// no code, header, table or helper with the GPU library.
//
// What it computes (SySTeC, Patel/Ahrens/Amarasinghe, CGO'25, arXiv 2406.09266):
//
//  * A symmetric tensor is invariant under every permutation of its indices
//    (Sec. 2.1, Definition "Symmetry"). Only canonical coordinates, whose
//    indices ascend, are stored (Sec. 2.1, Definition "Canonical"; the upper
//    triangle is the chosen one).
//  * Every stored entry (c, v) therefore stands for the value v at every
//    DISTINCT permutation of its index tuple c. There are N!/prod(m!) of them
//    when the tuple has runs of equal values of lengths m (Sec. 3.1, the
//    paragraph after the TTM listing). A stored diagonal value is not
//    pre-scaled: it is the value of each coordinate of its orbit (Fig. on
//    SSYMV, the i == j branch performs one update with the stored value).
//  * The full tensor is T[p] = sum over entries e with p in Perm(c_e) of v_e.
//    Duplicate canonical tuples add.
//  * The kernels are the plain definitions over T:
//      SSYMV   y[i]     = sum_j A[i,j] x[j]                     (Sec. 5.2.1)
//      SYPRD   s        = sum_{i,j} x[i] A[i,j] x[j]            (Sec. 5.2.3)
//      MTTKRP  C[i,r]   = sum_{k2..kN} T[i,k2..kN] prod_t B[kt,r]
//                                                              (Sec. 5.2.6)
//
// The oracle never uses a multiplicity formula or a coefficient table to form
// a result. It walks the distinct permutations of each stored tuple with
// std::next_permutation (which visits every distinct arrangement of a multiset
// exactly once, in lexicographic order, starting from the sorted one) and
// applies the plain definition to each. Independently it computes
// N!/prod(m!) from the run lengths in integer arithmetic and fails if the two
// counts differ.
//
// Beyond the three kernels above, the oracle defines the kernels built next to
// them, again as plain definitions over the expanded tensor:
//      Bellman-Ford  y[i]   = min_j (A[i,j] + d[j])  over stored coordinates
//                                                              (Sec. 5.2.2)
//      TTM           C[j,l,r] = sum_k A[k,j,l] B[k,r]          (Sec. 5.2.5)
//      MTTKRP of a partially symmetric tensor (Sec. 2.1, "Partial Symmetry"):
//                    the tensor is invariant only under permutations inside
//                    each part of a partition of its slots, so a stored entry
//                    stands for every arrangement obtained by permuting each
//                    part separately (the product of the parts' distinct
//                    permutations), and C[i,r] = sum T[i,k2..kN] prod_t
//                    F_{part(t)}[kt,r] with one factor matrix per part.
//
// Indices are 0-based (the paper's listings are Julia, 1-based). All values
// are FP64; FP32 and BF16 inputs convert to FP64 exactly.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include <omp.h>

extern "C" {

enum { ORACLE_OK = 0, ORACLE_EINVAL = 1, ORACLE_ECOUNT = 2 };

// Counters reported by every oracle call.
typedef struct {
  int64_t entries;        // stored entries visited
  int64_t effective_nnz;  // sum over entries of the number of distinct permutations
  int64_t noncanonical;   // entries whose stored tuple did not ascend (sorted, same orbit)
  int64_t hist[16];       // entries per equality pattern of the sorted tuple:
                          // bit t (t = 0..N-2) set when c[t] == c[t+1]
} oracle_counts;

}  // extern "C"

namespace {

const int kMaxOrder = 5;

int64_t factorial(int n) {
  int64_t f = 1;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

// N! / prod(m!) over the runs of equal values of a sorted tuple, in integers.
int64_t distinct_perm_count(const int32_t* c, int n) {
  int64_t denom = 1;
  int run = 1;
  for (int t = 1; t <= n; ++t) {
    if (t < n && c[t] == c[t - 1]) {
      ++run;
    } else {
      denom *= factorial(run);
      run = 1;
    }
  }
  return factorial(n) / denom;
}

void reset(oracle_counts* k) { std::memset(k, 0, sizeof(*k)); }

// Sorts one stored tuple into ascending order, counting it if it was not.
// Records its equality pattern. Returns false on an out-of-range index.
bool prepare_tuple(int32_t* c, int n, int64_t dim, oracle_counts* k) {
  for (int t = 0; t < n; ++t)
    if (c[t] < 0 || c[t] >= dim) return false;
  bool ascending = true;
  for (int t = 1; t < n; ++t)
    if (c[t - 1] > c[t]) ascending = false;
  if (!ascending) {
    std::sort(c, c + n);
    k->noncanonical += 1;
  }
  int pattern = 0;
  for (int t = 0; t + 1 < n; ++t)
    if (c[t] == c[t + 1]) pattern |= 1 << t;
  k->hist[pattern] += 1;
  k->entries += 1;
  return true;
}

// Visits every distinct permutation p of the sorted tuple c and calls f(p).
// Returns the number visited, or -1 if it differs from N!/prod(m!).
template <class F>
int64_t for_each_distinct_permutation(const int32_t* c, int n, F&& f) {
  int32_t p[kMaxOrder];
  std::memcpy(p, c, sizeof(int32_t) * n);
  int64_t visited = 0;
  do {
    f(p);
    ++visited;
  } while (std::next_permutation(p, p + n));
  if (visited != distinct_perm_count(c, n)) return -1;
  return visited;
}

// The SSYMV updates of stored rows [i0, i1), added into y; counts accumulate.
int ssymv_rows(int64_t n, int64_t i0, int64_t i1, const int32_t* rowptr, const int32_t* col,
               const double* val, const double* x, const uint8_t* row_mask, double* y,
               oracle_counts* counts) {
  for (int64_t i = i0; i < i1; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return ORACLE_EINVAL;
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      int32_t c[2] = {(int32_t)i, col[q]};
      if (!prepare_tuple(c, 2, n, counts)) return ORACLE_EINVAL;
      const double a = val[q];
      int64_t k = for_each_distinct_permutation(c, 2, [&](const int32_t* p) {
        if (row_mask && !row_mask[p[0]]) return;
        y[p[0]] += a * x[p[1]];
      });
      if (k < 0) return ORACLE_ECOUNT;
      counts->effective_nnz += k;
    }
  }
  return ORACLE_OK;
}

}  // namespace

extern "C" {

// Expansion only: counts, histogram and (optionally) the expanded coordinate
// list. idx is entry-major: idx[e*order + t]. If coords is not NULL it
// receives the expanded coordinates (entry-major, order ints each) up to cap
// coordinates; perm_count (optional) receives the per-entry count.
int oracle_expand(int order, int64_t dim, int64_t nnz, const int32_t* idx,
                  int64_t* perm_count, int32_t* coords, int64_t cap,
                  oracle_counts* counts) {
  if (order < 1 || order > kMaxOrder || dim < 1 || nnz < 0 || !counts) return ORACLE_EINVAL;
  reset(counts);
  int64_t written = 0;
  for (int64_t e = 0; e < nnz; ++e) {
    int32_t c[kMaxOrder];
    std::memcpy(c, idx + e * order, sizeof(int32_t) * order);
    if (!prepare_tuple(c, order, dim, counts)) return ORACLE_EINVAL;
    int64_t k = for_each_distinct_permutation(c, order, [&](const int32_t* p) {
      if (coords && written < cap)
        std::memcpy(coords + written * order, p, sizeof(int32_t) * order);
      ++written;
    });
    if (k < 0) return ORACLE_ECOUNT;
    if (perm_count) perm_count[e] = k;
    counts->effective_nnz += k;
  }
  return ORACLE_OK;
}

// MTTKRP of order N over the expanded tensor (Sec. 5.2.6):
//   C[p_s, r] += v * prod_{t != s} B[p_t, r]   for every distinct permutation p
// with s = out_slot (0 gives the paper's mode-1 output; every slot gives the
// same C for a symmetric tensor). idx is entry-major (nnz x order), B is
// dim x R row-major, C (dim x R row-major) is overwritten. If row_mask is not
// NULL, only rows i with row_mask[i] != 0 are computed (the others stay 0);
// the expansion and its counts still cover every entry.
int oracle_mttkrp(int order, int64_t dim, int64_t nnz, const int32_t* idx,
                  const double* val, int64_t R, const double* B, int out_slot,
                  const uint8_t* row_mask, double* C, oracle_counts* counts) {
  if (order < 1 || order > kMaxOrder || dim < 1 || nnz < 0 || R < 1 || out_slot < 0 ||
      out_slot >= order || !C || !counts)
    return ORACLE_EINVAL;
  reset(counts);
  std::fill(C, C + dim * R, 0.0);
  for (int64_t e = 0; e < nnz; ++e) {
    int32_t c[kMaxOrder];
    std::memcpy(c, idx + e * order, sizeof(int32_t) * order);
    if (!prepare_tuple(c, order, dim, counts)) return ORACLE_EINVAL;
    const double v = val[e];
    int64_t k = for_each_distinct_permutation(c, order, [&](const int32_t* p) {
      const int64_t out = p[out_slot];
      if (row_mask && !row_mask[out]) return;
      double* crow = C + out * R;
      for (int64_t r = 0; r < R; ++r) {
        double prod = v;
        for (int t = 0; t < order; ++t)
          if (t != out_slot) prod *= B[p[t] * R + r];
        crow[r] += prod;
      }
    });
    if (k < 0) return ORACLE_ECOUNT;
    counts->effective_nnz += k;
  }
  return ORACLE_OK;
}

// SSYMV over the expanded matrix (Sec. 5.2.1): y[p1] += A[p1,p2] * x[p2] for
// both distinct permutations of a stored (i, j), one when i == j. The matrix
// comes as CSR of the stored triangle: row i holds entries (i, col[k]).
// y is overwritten. row_mask as in oracle_mttkrp.
int oracle_ssymv(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                 const double* x, const uint8_t* row_mask, double* y, oracle_counts* counts) {
  if (n < 1 || !rowptr || !y || !counts) return ORACLE_EINVAL;
  reset(counts);
  std::fill(y, y + n, 0.0);
  if (rowptr[0] != 0) return ORACLE_EINVAL;
  return ssymv_rows(n, 0, n, rowptr, col, val, x, row_mask, y, counts);
}

// SYPRD over the expanded matrix (Sec. 5.2.3): s = sum over every distinct
// permutation p of every stored entry of x[p1] * A[p1,p2] * x[p2].
// abs_s receives the same sum of absolute values (an error scale for a result
// that can cancel to zero).
int oracle_syprd(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                 const double* x, double* s, double* abs_s, oracle_counts* counts) {
  if (n < 1 || !rowptr || !s || !counts) return ORACLE_EINVAL;
  reset(counts);
  double acc = 0.0, acc_abs = 0.0;
  if (rowptr[0] != 0) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return ORACLE_EINVAL;
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      int32_t c[2] = {(int32_t)i, col[q]};
      if (!prepare_tuple(c, 2, n, counts)) return ORACLE_EINVAL;
      const double a = val[q];
      int64_t k = for_each_distinct_permutation(c, 2, [&](const int32_t* p) {
        double term = x[p[0]] * a * x[p[1]];
        acc += term;
        acc_abs += std::fabs(term);
      });
      if (k < 0) return ORACLE_ECOUNT;
      counts->effective_nnz += k;
    }
  }
  *s = acc;
  if (abs_s) *abs_s = acc_abs;
  return ORACLE_OK;
}

// Rounds FP32 values to bfloat16 (8 significant bits, FP32's exponent range)
// with round-to-nearest, ties to even, and returns them widened to FP64.
// Written from the number format's definition: the result is the multiple of
// the bfloat16 unit in the last place nearest to the input. Inputs must be
// finite and within bfloat16's range.
int oracle_round_bf16(const float* in, double* out, int64_t n) {
  if (n < 0) return ORACLE_EINVAL;
  for (int64_t q = 0; q < n; ++q) {
    const double v = in[q];
    if (v == 0.0 || !std::isfinite(v)) {
      out[q] = v;
      continue;
    }
    int e;
    std::frexp(v, &e);  // v = m * 2^e, 0.5 <= |m| < 1
    // Unit in the last place of an 8-bit significand; below the smallest
    // normal (2^-126) the spacing stays 2^-133.
    int ulp_exp = std::max(e - 8, -133);
    double scaled = std::ldexp(v, -ulp_exp);  // exact: only the exponent changes
    double r = std::nearbyint(scaled);        // default mode: nearest, ties to even
    out[q] = std::ldexp(r, ulp_exp);
  }
  return ORACLE_OK;
}

}  // extern "C"

// ---- all-core variants ----------------------------------------------------
// The same loops over a static partition of the stored entries into
// `threads` contiguous ranges: each thread runs the single-threaded oracle on
// its range into a private FP64 output, and the private outputs are added in
// thread order, element by element. Deterministic for a fixed thread count;
// the result differs from the single-threaded one only in the order of FP64
// additions. Counts are summed. threads <= 0 takes every core OpenMP sees.

namespace {

int resolve_threads(int threads) { return threads > 0 ? threads : omp_get_max_threads(); }

void add_counts(oracle_counts* into, const oracle_counts& k) {
  into->entries += k.entries;
  into->effective_nnz += k.effective_nnz;
  into->noncanonical += k.noncanonical;
  for (int m = 0; m < 16; ++m) into->hist[m] += k.hist[m];
}

// out[q] = sum over threads t (in order) of part[t][q], q < len
void sum_in_thread_order(const std::vector<std::vector<double>>& part, double* out, int64_t len) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < len; ++q) {
    double s = 0.0;
    for (const auto& p : part) s += p[q];
    out[q] = s;
  }
}

}  // namespace

extern "C" {

int oracle_mttkrp_mt(int order, int64_t dim, int64_t nnz, const int32_t* idx,
                     const double* val, int64_t R, const double* B, int out_slot,
                     const uint8_t* row_mask, double* C, oracle_counts* counts, int threads) {
  const int T = resolve_threads(threads);
  if (T <= 1)
    return oracle_mttkrp(order, dim, nnz, idx, val, R, B, out_slot, row_mask, C, counts);
  if (order < 1 || order > kMaxOrder || dim < 1 || nnz < 0 || R < 1 || !C || !counts)
    return ORACLE_EINVAL;
  std::vector<std::vector<double>> part(T, std::vector<double>(dim * R));
  std::vector<oracle_counts> kc(T);
  std::vector<int> rc(T, ORACLE_OK);
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    const int64_t e0 = nnz * t / T, e1 = nnz * (t + 1) / T;
    rc[t] = oracle_mttkrp(order, dim, e1 - e0, idx + e0 * order, val + e0, R, B, out_slot,
                          row_mask, part[t].data(), &kc[t]);
  }
  reset(counts);
  for (int t = 0; t < T; ++t) {
    if (rc[t] != ORACLE_OK) return rc[t];
    add_counts(counts, kc[t]);
  }
  sum_in_thread_order(part, C, dim * R);
  return ORACLE_OK;
}

// Rows are split so that each thread gets about nnz / T stored entries.
int oracle_ssymv_mt(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                    const double* x, const uint8_t* row_mask, double* y, oracle_counts* counts,
                    int threads) {
  const int T = resolve_threads(threads);
  if (T <= 1) return oracle_ssymv(n, rowptr, col, val, x, row_mask, y, counts);
  if (n < 1 || !rowptr || !y || !counts || rowptr[0] != 0) return ORACLE_EINVAL;
  const int64_t nnz = rowptr[n];
  std::vector<int64_t> r0(T + 1, n);
  r0[0] = 0;
  for (int t = 1; t < T; ++t)
    r0[t] = std::lower_bound(rowptr, rowptr + n + 1, nnz * t / T) - rowptr;
  std::vector<std::vector<double>> part(T, std::vector<double>(n));
  std::vector<oracle_counts> kc(T);
  std::vector<int> rc(T, ORACLE_OK);
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    reset(&kc[t]);
    rc[t] = ssymv_rows(n, r0[t], r0[t + 1], rowptr, col, val, x, row_mask, part[t].data(), &kc[t]);
  }
  reset(counts);
  for (int t = 0; t < T; ++t) {
    if (rc[t] != ORACLE_OK) return rc[t];
    add_counts(counts, kc[t]);
  }
  sum_in_thread_order(part, y, n);
  return ORACLE_OK;
}

int oracle_threads(void) { return omp_get_max_threads(); }

}  // extern "C"

// ---- kernels beyond SSYMV, SYPRD and MTTKRP ---------------------------------

namespace {

// Visits every arrangement of c obtained by permuting, independently, the
// slots of each part (parts are consecutive slot ranges start[q] ..
// start[q] + size[q] - 1, each sorted ascending on entry) and calls f(p).
template <class F>
void for_each_part_arrangement(int32_t* p, int q, int nparts, const int* start, const int* size,
                               int64_t* visited, F& f) {
  if (q == nparts) {
    f(p);
    ++*visited;
    return;
  }
  // std::next_permutation returns false once it has wrapped back to the
  // ascending order, so the part is left as it was found
  do {
    for_each_part_arrangement(p, q + 1, nparts, start, size, visited, f);
  } while (std::next_permutation(p + start[q], p + start[q] + size[q]));
}

}  // namespace

extern "C" {

// Bellman-Ford update (Sec. 5.2.2), the (min, +) form of SSYMV: for every
// distinct permutation p of every stored (i, j, a), y[p1] = min(y[p1],
// a + d[p2]). Starts from +infinity (the identity of min), so an index with
// no stored coordinate stays +infinity. Matrix as for oracle_ssymv.
int oracle_bellman_ford(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                        const double* d, double* y, oracle_counts* counts) {
  if (n < 1 || !rowptr || !y || !d || !counts) return ORACLE_EINVAL;
  reset(counts);
  std::fill(y, y + n, std::numeric_limits<double>::infinity());
  if (rowptr[0] != 0) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return ORACLE_EINVAL;
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      int32_t c[2] = {(int32_t)i, col[q]};
      if (!prepare_tuple(c, 2, n, counts)) return ORACLE_EINVAL;
      const double a = val[q];
      int64_t k = for_each_distinct_permutation(c, 2, [&](const int32_t* p) {
        y[p[0]] = std::min(y[p[0]], a + d[p[1]]);
      });
      if (k < 0) return ORACLE_ECOUNT;
      counts->effective_nnz += k;
    }
  }
  return ORACLE_OK;
}

// TTM of a fully symmetric 3-index tensor A (Sec. 5.2.5): C[i,j,l] =
// sum_k A[k,j,l] * B[k,i], with i the column of B (r below). For every
// distinct permutation p = (k, j, l) of every stored tuple:
// C[j][l][r] += v * B[k][r]. C is dim x dim x R with r fastest, overwritten.
int oracle_ttm3(int64_t dim, int64_t nnz, const int32_t* idx, const double* val, int64_t R,
                const double* B, double* C, oracle_counts* counts) {
  if (dim < 1 || nnz < 0 || R < 1 || !C || !counts) return ORACLE_EINVAL;
  reset(counts);
  std::fill(C, C + dim * dim * R, 0.0);
  for (int64_t e = 0; e < nnz; ++e) {
    int32_t c[3];
    std::memcpy(c, idx + e * 3, sizeof(c));
    if (!prepare_tuple(c, 3, dim, counts)) return ORACLE_EINVAL;
    const double v = val[e];
    int64_t k = for_each_distinct_permutation(c, 3, [&](const int32_t* p) {
      double* out = C + (static_cast<int64_t>(p[1]) * dim + p[2]) * R;
      const double* b = B + static_cast<int64_t>(p[0]) * R;
      for (int64_t r = 0; r < R; ++r) out[r] += v * b[r];
    });
    if (k < 0) return ORACLE_ECOUNT;
    counts->effective_nnz += k;
  }
  return ORACLE_OK;
}

// MTTKRP of a partially symmetric tensor. The slots form nparts consecutive
// parts of sizes part_size[0..nparts-1] (summing to order); the tensor is
// symmetric within each part only (Sec. 2.1, Definition "Partial
// Symmetry"), and a coordinate is canonical when its indices ascend inside
// every part (Definition "Canonical"). F holds one dim x R factor matrix per
// part (F + q*dim*R). For every arrangement p of every stored tuple (each
// part permuted on its own, distinct arrangements only):
//   C[p_1][r] += v * prod_{t >= 2} F_{part(t)}[p_t][r]
// (the output is mode 1, in part 0). A tuple whose part does not ascend is
// sorted inside that part (same orbit) and counted as non-canonical. The
// visited count must equal the product of the parts' N_q!/prod(m!) counts.
// hist records the equality pattern of slots adjacent inside one part.
int oracle_mttkrp_partial(int order, int nparts, const int32_t* part_size, int64_t dim,
                          int64_t nnz, const int32_t* idx, const double* val, int64_t R,
                          const double* F, double* C, oracle_counts* counts) {
  if (order < 1 || order > kMaxOrder || nparts < 1 || nparts > order || !part_size || dim < 1 ||
      nnz < 0 || R < 1 || !F || !C || !counts)
    return ORACLE_EINVAL;
  int start[kMaxOrder], size[kMaxOrder], part_of[kMaxOrder];
  int sum = 0;
  for (int q = 0; q < nparts; ++q) {
    if (part_size[q] < 1) return ORACLE_EINVAL;
    start[q] = sum;
    size[q] = part_size[q];
    for (int t = sum; t < sum + size[q] && t < kMaxOrder; ++t) part_of[t] = q;
    sum += size[q];
  }
  if (sum != order) return ORACLE_EINVAL;
  reset(counts);
  std::fill(C, C + dim * R, 0.0);
  for (int64_t e = 0; e < nnz; ++e) {
    int32_t c[kMaxOrder];
    std::memcpy(c, idx + e * order, sizeof(int32_t) * order);
    bool canonical = true;
    for (int t = 0; t < order; ++t)
      if (c[t] < 0 || c[t] >= dim) return ORACLE_EINVAL;
    for (int q = 0; q < nparts; ++q) {
      for (int t = start[q] + 1; t < start[q] + size[q]; ++t)
        if (c[t - 1] > c[t]) canonical = false;
      std::sort(c + start[q], c + start[q] + size[q]);
    }
    if (!canonical) counts->noncanonical += 1;
    int pattern = 0;
    for (int t = 0; t + 1 < order; ++t)
      if (part_of[t] == part_of[t + 1] && c[t] == c[t + 1]) pattern |= 1 << t;
    counts->hist[pattern] += 1;
    counts->entries += 1;
    int64_t expected = 1;
    for (int q = 0; q < nparts; ++q) expected *= distinct_perm_count(c + start[q], size[q]);
    const double v = val[e];
    int32_t p[kMaxOrder];
    std::memcpy(p, c, sizeof(int32_t) * order);
    int64_t visited = 0;
    auto update = [&](const int32_t* a) {
      double* crow = C + static_cast<int64_t>(a[0]) * R;
      for (int64_t r = 0; r < R; ++r) {
        double prod = v;
        for (int t = 1; t < order; ++t)
          prod *= F[(static_cast<int64_t>(part_of[t]) * dim + a[t]) * R + r];
        crow[r] += prod;
      }
    };
    for_each_part_arrangement(p, 0, nparts, start, size, &visited, update);
    if (visited != expected) return ORACLE_ECOUNT;
    counts->effective_nnz += visited;
  }
  return ORACLE_OK;
}

}  // extern "C"
