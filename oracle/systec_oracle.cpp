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
// Indices are 0-based (the paper's listings are Julia, 1-based). All values
// are FP64; FP32 and BF16 inputs convert to FP64 exactly.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

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
  for (int64_t i = 0; i < n; ++i) {
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
