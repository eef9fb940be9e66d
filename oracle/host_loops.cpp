// The method's symmetric loops on one host core, in FP64: the benchmark's
// CPU analog of the paper's symmetric-against-naive comparison.
//
// TEST INFRASTRUCTURE (benchmark baseline) ONLY. Only the test suite and the
// CPU-baseline leg of the benchmark load this. It is not the oracle and
// decides no parity question: the oracle (systec_oracle.cpp) defines the
// kernels over the expanded tensor; these loops compute the same results
// from the canonical entries alone, and the tests pin them to the oracle.
// It shares no code with the GPU library or with the oracle.
//
// SySTeC, arXiv 2406.09266:
//  * SSYMV over the stored upper triangle (Sec. 3.1): each stored a =
//    A[i,j], i <= j, gives y[i] += a x[j] and, when i < j, y[j] += a x[i].
//  * MTTKRP over canonical tuples (Sec. 4.2.5, 4.2.7, 5.2.6): the distinct
//    permutations of a tuple with value v in the first slot number
//    (N-1)! m_v / prod(m!) (m_v the copies of v, m the run lengths), and
//    each contributes val * prod of B over the tuple with one copy of v
//    removed, so every distinct value v of the tuple adds that count times
//    val * prod_{s != t} B[c_s, :] to C[v, :] (t the first slot holding v).
#include <stdint.h>

#include <cstring>

extern "C" {

// y = A x; rowptr/col the canonical CSR (col >= row, ascending in a row).
// Returns 1 on an invalid argument or index.
int host_ssymv_canonical(int64_t n, const int32_t* rowptr, const int32_t* col,
                         const double* val, const double* x, double* y) {
  if (n < 0 || !rowptr || (n > 0 && (!x || !y))) return 1;
  for (int64_t i = 0; i < n; ++i) y[i] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int64_t j = col[e];
      if (j < i || j >= n) return 1;
      y[i] += val[e] * x[j];
      if (j != i) y[j] += val[e] * x[i];
    }
  }
  return 0;
}

// C (dim x R, row-major) = MTTKRP of the symmetric tensor of `nnz`
// canonical tuples; idx entry-major (idx[e * order + t], ascending in t),
// B dim x R row-major. Returns 1 on an invalid argument or index.
int host_mttkrp_canonical(int order, int64_t dim, int64_t nnz, const int32_t* idx,
                          const double* val, const double* B, int64_t R, double* C) {
  if (order < 2 || order > 5 || dim < 0 || nnz < 0 || R < 1 || !C) return 1;
  for (int64_t k = 0; k < dim * R; ++k) C[k] = 0.0;
  int64_t fact[6] = {1, 1, 2, 6, 24, 120};
  for (int64_t e = 0; e < nnz; ++e) {
    const int32_t* c = idx + e * order;
    for (int t = 0; t < order; ++t) {
      if (c[t] < 0 || c[t] >= dim || (t > 0 && c[t] < c[t - 1])) return 1;
    }
    // run lengths: prod(m!) and, per slot, the run length of its value
    int64_t denom = 1;
    int run_len[5] = {0, 0, 0, 0, 0};
    for (int t = 0; t < order;) {
      int u = t;
      while (u < order && c[u] == c[t]) ++u;
      denom *= fact[u - t];
      for (int q = t; q < u; ++q) run_len[q] = u - t;
      t = u;
    }
    for (int t = 0; t < order; ++t) {
      if (t > 0 && c[t] == c[t - 1]) continue;  // one update per distinct value
      const double count = static_cast<double>(fact[order - 1] * run_len[t]) /
                           static_cast<double>(denom);  // an integer
      double* out = C + static_cast<int64_t>(c[t]) * R;
      for (int64_t r = 0; r < R; ++r) {
        double p = count * val[e];
        for (int s = 0; s < order; ++s)
          if (s != t) p *= B[static_cast<int64_t>(c[s]) * R + r];
        out[r] += p;
      }
    }
  }
  return 0;
}

}  // extern "C"
