/*
 * systec.h - symmetric sparse tensor kernels on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates kernels whose sparse operand is a fully symmetric
 * tensor stored by its canonical coordinates only (indices ascending, the
 * upper triangle for a matrix; SySTeC, arXiv 2406.09266, Sec. 2.1,
 * definitions "Symmetry" and "Canonical"). Each stored entry is expanded on
 * the fly into its distinct index permutations: one read of a stored value
 * serves every output it contributes to (Sec. 3.1, "reusing canonical
 * reads"), weighted by how many distinct permutations land on the same output
 * (Sec. 3.2.2, invisible output symmetry; Sec. 4.2.5 and 4.2.7). The result is
 * the plain kernel over the full symmetric tensor.
 *
 * Conventions for every entry point:
 *  - Return value: SYSTEC_OK (0) or a systec_status code. Nothing throws or
 *    aborts across this interface. systec_last_error() gives a message for
 *    the last failure on the calling thread.
 *  - Indices are 0-based int32. Counts are int64 but must stay below 2^31.
 *  - Pointers marked "device" address GPU memory (hipMalloc, torch CUDA
 *    tensors); "host" pointers address CPU memory. The caller owns every
 *    buffer it passes. Calls are asynchronous on `stream` (a hipStream_t;
 *    NULL is the default stream): buffers must stay valid until the stream's
 *    work completes. Output buffers are overwritten (the library zeroes them
 *    on `stream`); there is no accumulate mode.
 *  - Arguments are checked on the host: a bad size, order, dtype or NULL
 *    pointer (other than for empty inputs) returns SYSTEC_EINVAL and launches
 *    nothing. The canonical form of the sparse operand is the caller's
 *    contract; systec_validate_* checks it on the device and
 *    systec_canonicalize_coo establishes it on the host. A HIP failure
 *    returns SYSTEC_EDEVICE with HIP's message.
 *  - Floating point: stored tensor values are FP32. Vectors and factor
 *    matrices are FP32 or BF16 (systec_dtype); BF16 values are widened
 *    exactly to FP32 in registers. Products and sums are FP32; outputs are
 *    accumulated with FP32 atomics, so their summation order (and last bits)
 *    varies between runs. Scalar results are reduced in FP64 at the end.
 */
#ifndef SYSTEC_H
#define SYSTEC_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SYSTEC_API __attribute__((visibility("default")))
#else
#define SYSTEC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SYSTEC_OK = 0,
  SYSTEC_EINVAL = 1,     /* bad argument (size, order, dtype, NULL pointer)   */
  SYSTEC_ENONCANON = 2,  /* sparse operand not in canonical form (validation) */
  SYSTEC_ENOMEM = 3,     /* device allocation failed                          */
  SYSTEC_EBUDGET = 4,    /* request can never fit the serving memory budget   */
  SYSTEC_EBUSY = 5,      /* serving queue full                                */
  SYSTEC_ETIMEOUT = 6,   /* wait timed out                                    */
  SYSTEC_ENOTFOUND = 7,  /* unknown tensor or request id                      */
  SYSTEC_EDEVICE = 8     /* HIP runtime or kernel launch failure              */
} systec_status;

/* Element type of a dense vector or factor matrix. */
typedef enum { SYSTEC_F32 = 0, SYSTEC_BF16 = 1 } systec_dtype;

/* A hipStream_t passed as an opaque pointer (torch: current_stream().cuda_stream). */
typedef void* systec_stream;

/* Message for the last failing call on this thread ("" if none). Never NULL. */
SYSTEC_API const char* systec_last_error(void);

/* Library version string. */
SYSTEC_API const char* systec_version(void);

/* ------------------------------------------------------------------------
 * SSYMV  y = A x  (Sec. 5.2.1: A symmetric sparse, x and y dense).
 *
 * A is given by its stored upper triangle in CSR (diagonal included):
 *   rowptr  device int32[n+1], rowptr[0] = 0, nondecreasing, rowptr[n] = nnz
 *   col     device int32[nnz], col >= row, ascending within a row, < n
 *   val     device float[nnz]
 * A stored off-diagonal a = A[i,j] (i < j) updates y[i] += a x[j] and
 * y[j] += a x[i]; a diagonal one updates y[i] += a x[i] (Sec. 3.1, the SSYMV
 * figure). The stored value of a diagonal entry is not pre-scaled.
 *   x       device, n elements of dtype xdt (F32 or BF16)
 *   y       device float[n], overwritten.
 * n >= 1, 0 <= nnz < 2^31. Errors: EINVAL, EDEVICE, ENOMEM.
 * From 2^18 stored entries (and up to 2^26 rows) the column-side updates
 * are binned by ranges of 16,384 columns and summed in LDS instead of sent
 * as device atomics; the call then allocates stream-ordered scratch
 * (hipMallocAsync, about 8 bytes per stored entry), freed on the stream
 * when the call's work is done.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_ssymv(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                 const float* val, const void* x, systec_dtype xdt, float* y,
                 systec_stream stream);

/* ------------------------------------------------------------------------
 * SYPRD  s = x^T A x  (Sec. 5.2.3; Sec. 3.2.2: an off-diagonal stored entry
 * contributes 2 x[i] a x[j], a diagonal one x[i] a x[i]).
 * A, x as for systec_ssymv. Per-block partial sums are FP32; the final sum
 * over blocks is FP64 on the device.
 *   out     device double[1], overwritten.
 * Errors: EINVAL, EDEVICE.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_syprd(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                 const float* val, const void* x, systec_dtype xdt, double* out,
                 systec_stream stream);

/* systec_syprd that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Arguments, result and errors as for
 * systec_syprd; the per-workgroup partials live in a fixed 1 MiB array of
 * the library, one per device, held until the process ends, so n + nnz may
 * be at most 536,870,912 (2^29; larger: SYSTEC_EINVAL, nothing launched).
 * Every call on a device uses that device's one array: calls that overlap
 * on one device (different streams, threads) race and must be serialized
 * by the caller. SYSTEC_VALIDATE is not applied here. */
SYSTEC_API int systec_syprd_noalloc(int64_t n, int64_t nnz, const int32_t* rowptr,
                                    const int32_t* col, const float* val, const void* x,
                                    systec_dtype xdt, double* out, systec_stream stream);

/* ------------------------------------------------------------------------
 * Bellman-Ford update  y[i] = min_j (A[i,j] + d[j])  (Sec. 5.2.2: A the
 * symmetric matrix of edge lengths, d the path lengths after k steps, y
 * after k + 1; the (min, +) form of SSYMV). The minimum runs over the
 * coordinates the full symmetric matrix stores: a stored a = A[i,j], i < j,
 * offers y[i] the value a + d[j] and y[j] the value a + d[i]; a diagonal one
 * offers y[i] the value a + d[i]. An index with no stored coordinate gets
 * +inf (the identity of min); to carry d[i] over, store a zero diagonal.
 * A as for systec_ssymv (stored values are the edge lengths, FP32);
 *   d       device float[n], finite or +inf
 *   y       device float[n], overwritten.
 * Each y[i] is the FP32 sum a + d of its minimizing coordinate, independent
 * of the order of the updates (the minima are taken exactly, on integer keys
 * that order like the values). Errors: EINVAL, EDEVICE.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_bellman_ford(int64_t n, int64_t nnz, const int32_t* rowptr,
                                   const int32_t* col, const float* val, const float* d,
                                   float* y, systec_stream stream);

/* ------------------------------------------------------------------------
 * Symmetric MTTKRP of order N = 3, 4, 5 (Sec. 5.2.6):
 *   C[i,r] = sum_{k2..kN} T[i,k2,..,kN] * B[k2,r] * ... * B[kN,r]
 * T is fully symmetric, given by its canonical entries in COO, structure of
 * arrays, sorted lexicographically (so grouped by the leading index):
 *   idx     host array of `order` device pointers; idx[t] is int32[nnz] and
 *           idx[0][e] <= idx[1][e] <= ... <= idx[order-1][e] < I
 *   val     device float[nnz]
 *   B       device I x R row-major, dtype bdt (F32 or BF16)
 *   C       device float I x R row-major, overwritten.
 * Each entry with value v updates, for every slot t that starts a run of
 * equal indices, C[idx[t][e], :] += coef * v * prod_{s != t} B[idx[s][e], :],
 * where coef = (number of distinct permutations of the tuple) * (run
 * length) / order. (Sec. 3.1: N!/m! assignments per read; Sec. 4.3, the 3-D
 * derivation and its split loop nests.)
 * order in {3,4,5}, I >= 1, R >= 1, 0 <= nnz < 2^31, I*R < 2^31.
 * Errors: EINVAL, EDEVICE.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_mttkrp(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                  const float* val, const void* B, systec_dtype bdt, int64_t R, float* C,
                  systec_stream stream);

/* ------------------------------------------------------------------------
 * TTM with visible output symmetry (Sec. 5.2.5; Sec. 3.2.1, visible output
 * symmetry): for a fully symmetric 3-index tensor T,
 *   C[j, l, r] = sum_k T[k, j, l] B[k, r]
 * T as canonical COO of order 3 (as for systec_mttkrp); B device I x R
 * (F32 or BF16); C device float I x I x R, row-major (r fastest), dense.
 * C is symmetric in (j, l): the call computes its canonical half, j <= l,
 * from the stored entries (an entry updates C[j, l, :] += v B[k, :] once per
 * distinct value k of its tuple, with (j, l) the other two indices in
 * ascending order) and, if mirror == 1, copies it to the other half (the
 * paper's post-processing loop); with mirror == 0 the entries with j > l are
 * left untouched. The canonical half is overwritten.
 * I >= 1, 1 <= R, I * R < 2^31, I * I * R < 2^40. Errors: EINVAL, EDEVICE.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_ttm(int64_t I, int64_t nnz, const int32_t* const* idx, const float* val,
                          const void* B, systec_dtype bdt, int64_t R, float* C, int mirror,
                          systec_stream stream);

/* ------------------------------------------------------------------------
 * MTTKRP of a partially symmetric tensor (Sec. 2.1, "Partial Symmetry"):
 * the `order` slots form `nparts` consecutive parts of sizes part_sizes[q]
 * (host int32[nparts], summing to order); the tensor is invariant under
 * permutations inside each part only and is given by its canonical entries
 * (indices ascending inside every part; the list sorted lexicographically).
 * Each part q has a factor matrix F[q] (host array of nparts device
 * pointers, each I x R of dtype fdt), and
 *   C[i, r] = sum T[i, k2, .., kN] prod_{t >= 2} F[part(t)][k_t, r]
 * (output mode 1, in part 0). An entry updates, for each slot t of part 0
 * that starts a run of equal indices, C[c_t, :] += coef * v * prod_{s != t}
 * F[part(s)][c_s, :], coef = (arrangements of part 0) * (run length) /
 * (size of part 0) * prod over the other parts of their arrangements. One
 * part of size `order` is the fully symmetric MTTKRP.
 *   C       device float I x R, overwritten.
 * order in {2..5}, I >= 1, R >= 1, I*R < 2^31. Errors: EINVAL, EDEVICE.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_mttkrp_partial(int order, int nparts, const int32_t* part_sizes, int64_t I,
                                     int64_t nnz, const int32_t* const* idx, const float* val,
                                     const void* const* F, systec_dtype fdt, int64_t R,
                                     float* C, systec_stream stream);

/* ------------------------------------------------------------------------
 * How the updates of the non-leading slots are resolved (all give the same
 * result up to FP32 summation order):
 *   SYSTEC_MTTKRP_AUTO     the library chooses from I, R and the dtype (and,
 *                          for a prepared tensor, the lengths of its runs)
 *   SYSTEC_MTTKRP_ATOMIC   canonical list; leading slot summed in registers
 *                          across a run of equal c1 (Sec. 4.2.8), the other
 *                          run-start slots by device FP32 atomics
 *   SYSTEC_MTTKRP_LDS      slot views of a prepared tensor with B staged in
 *                          LDS: all of B with one lane per view entry when
 *                          I * R elements fit one workgroup's LDS (160 KiB:
 *                          I = 5,000 at R = 16 in BF16), R is 16 or 32 (or
 *                          8 in BF16), B is 16-byte aligned and the tensor
 *                          holds at least 64 entries per index; else column
 *                          slices of B (a slice of one 16-byte vector per
 *                          row, 8 BF16 or 4 FP32 columns, must fit: with
 *                          160 KiB that is I <= 10,220); otherwise EINVAL
 *   SYSTEC_MTTKRP_VIEWS    slot views of a prepared tensor (systec_mttkrp_t
 *                          only; EINVAL for the one-shot call)
 * ---------------------------------------------------------------------- */
typedef enum {
  SYSTEC_MTTKRP_AUTO = 0,
  SYSTEC_MTTKRP_ATOMIC = 1,
  SYSTEC_MTTKRP_LDS = 2,
  SYSTEC_MTTKRP_VIEWS = 3
} systec_mttkrp_algo;

/* The algorithm AUTO runs for this shape: *algo receives ATOMIC for a
 * one-shot call (prepared == 0); for a prepared tensor LDS when all of B
 * fits one workgroup's LDS with R 16 or 32 (or 8 in BF16), else VIEWS. A
 * prepared tensor with fewer than 64 entries per index, or a B that is not
 * 16-byte aligned, runs the views under AUTO even where LDS is reported.
 * Errors: EINVAL (NULL algo, I or R out of range, bad dtype). */
SYSTEC_API int systec_mttkrp_choose(int64_t I, systec_dtype bdt, int64_t R, int prepared,
                                    systec_mttkrp_algo* algo);

/* systec_mttkrp with an explicit algorithm (systec_mttkrp is AUTO; only
 * AUTO and ATOMIC apply to the one-shot call). */
SYSTEC_API int systec_mttkrp_ex(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                                const float* val, const void* B, systec_dtype bdt, int64_t R,
                                float* C, systec_mttkrp_algo algo, systec_stream stream);

/* ------------------------------------------------------------------------
 * Comparison kernels without symmetry (the paper's baseline is the same
 * kernel over the full tensor; Sec. 5.2, results normalized to it).
 *
 * systec_spmv_csr: y = A x for a general CSR matrix (full, not a triangle);
 *   arguments as for systec_ssymv without the col >= row condition.
 * systec_mttkrp_full: C[i,:] = sum over the listed (not symmetric) entries
 *   of v * prod_{t>=1} B[idx[t][e], :], output row idx[0][e]. idx[0] must be
 *   nondecreasing (grouped by output row); other slots are unconstrained.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_spmv_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                    const float* val, const void* x, systec_dtype xdt, float* y,
                    systec_stream stream);
SYSTEC_API int systec_mttkrp_full(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                       const float* val, const void* B, systec_dtype bdt, int64_t R, float* C,
                       systec_stream stream);

/* ------------------------------------------------------------------------
 * Expansion into the full (non-symmetric) tensor, for the comparison
 * kernels. Setup work, not part of a timed kernel.
 *
 * systec_expand_csr_size / systec_expand_csr: from the stored upper triangle
 *   (as for systec_ssymv) build the full CSR of A = U + U^T - diag(U).
 *   *full_nnz (host) receives 2*nnz - (number of diagonal entries). The
 *   caller allocates full_rowptr int32[n+1], full_col int32[full_nnz],
 *   full_val float[full_nnz] (device). Columns within a row are in no
 *   particular order. Synchronizes `stream`.
 * systec_expand_coo_size / systec_expand_coo: from canonical COO (as for
 *   systec_mttkrp) write every distinct permutation of every entry, grouped
 *   by the first index (rows ascending; order within a row unspecified).
 *   *full_nnz (host) receives the number of expanded entries. out_idx is a
 *   host array of `order` device int32[full_nnz] pointers; out_val device
 *   float[full_nnz]. Synchronizes `stream`.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_expand_csr_size(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                           int64_t* full_nnz, systec_stream stream);
SYSTEC_API int systec_expand_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                      const float* val, int32_t* full_rowptr, int32_t* full_col,
                      float* full_val, systec_stream stream);
SYSTEC_API int systec_expand_coo_size(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                           int64_t* full_nnz, systec_stream stream);
SYSTEC_API int systec_expand_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                      const float* val, int32_t* const* out_idx, float* out_val,
                      systec_stream stream);

/* ------------------------------------------------------------------------
 * Expansion statistics (integer, exact): for canonical COO (order 2..5),
 * hist[m] (host int64[16]) receives the number of entries whose sorted tuple
 * has equality pattern m (bit t set when idx[t] == idx[t+1]);
 * *effective_nnz (host) receives the sum over entries of the number of
 * distinct permutations. Synchronizes `stream`.
 * For order 2, pass the row index of every entry in idx[0] and the column
 * in idx[1]. Errors: EINVAL, EDEVICE.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_expansion_stats(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                           int64_t* hist, int64_t* effective_nnz, systec_stream stream);

/* ------------------------------------------------------------------------
 * Validation of the canonical form on the device. Returns SYSTEC_OK if it
 * holds, SYSTEC_ENONCANON (with a message naming the first kind of
 * violation found) if not. Synchronizes `stream`.
 * systec_validate_csr_upper: rowptr as documented, 0 <= col < n, col >= row,
 *   columns strictly ascending within each row.
 * systec_validate_coo: indices < I, each tuple ascending, the list strictly
 *   increasing in lexicographic order (sorted, no duplicate tuples).
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_validate_csr_upper(int64_t n, int64_t nnz, const int32_t* rowptr,
                              const int32_t* col, systec_stream stream);
SYSTEC_API int systec_validate_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                        systec_stream stream);

/* ------------------------------------------------------------------------
 * Host helper: brings a COO list (host memory, structure of arrays, any
 * order) into canonical form in place: sorts each tuple, sorts the list
 * lexicographically and sums duplicate tuples. *nnz_out receives the new
 * length (entries beyond it are unspecified). val is host double.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_canonicalize_coo(int order, int64_t nnz, int32_t* const* idx, double* val,
                            int64_t* nnz_out);

/* ------------------------------------------------------------------------
 * Quantization of FP32 to BF16 with round-to-nearest-even, on the device
 * (the served precision form stores vectors and factors in BF16).
 *   in device float[n], out device uint16[n] (BF16 bit patterns).
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_quantize_bf16(const float* in, uint16_t* out, int64_t n, systec_stream stream);

/* ------------------------------------------------------------------------
 * Prepared operands. A symmetric operand can be rearranged once on the
 * device into a layout that turns the scattered output updates into
 * segmented reductions (the data rearrangement the paper keeps outside its
 * timings, Sec. 5.2, and the symmetry-aware storage it names as future work,
 * Sec. 7). The canonical entries are kept, only reordered:
 *  - matrix: rows cut into panels of 8192 rows; inside a panel the stored
 *    entries are sorted by (column, row). systec_ssymv_t keeps the panel's
 *    row sums in LDS and reduces the column side by segments.
 *  - tensor of order 3..5: one slot view per index slot t, holding the
 *    entries whose slot t starts a run of equal indices, sorted by their
 *    slot-t index. systec_mttkrp_t reduces every view by segments.
 * The handle owns a device copy (systec_tensor_info reports its bytes); the
 * caller's buffers may be freed after create returns. Create validates the
 * canonical form on the device (SYSTEC_ENONCANON if it does not hold),
 * synchronizes `stream`, and returns SYSTEC_ENOMEM if the copy does not fit.
 * The handle may be used from any stream of the device it was created on.
 * The handle holds the work buffers its calls need (SYPRD's per-chunk
 * partials; for a relabeled matrix the input and output in the stored
 * order), so no call allocates; calls that use them and share the handle
 * are ordered on the device (each waits for the previous one's work, on
 * whatever stream it ran).
 * ---------------------------------------------------------------------- */
typedef struct systec_tensor systec_tensor;

SYSTEC_API int systec_tensor_create_csr(int64_t n, int64_t nnz, const int32_t* rowptr,
                                        const int32_t* col, const float* val,
                                        systec_stream stream, systec_tensor** out);
/* systec_tensor_create_csr with the vertex order chosen by the caller.
 * relabel = 1 stores the matrix with its vertices ordered by descending
 * degree (a symmetric permutation P A P^T, ties in vertex order): the
 * high-degree vertices then share panels and columns, and the column-side
 * updates of systec_ssymv_t merge into fewer cache lines; each call then
 * permutes x in and y out (two gathers of n elements, inside the call, on
 * its stream, through two n-element work vectors that the handle holds, so
 * that a call allocates nothing). relabel = 0 keeps the order
 * (what systec_tensor_create_csr does); relabel = -1 relabels when the
 * largest degree exceeds 8 times the mean (power-law graphs). Anything else
 * is SYSTEC_EINVAL. A server serves a relabeled matrix too: each of its
 * requests then holds two more n-element vectors, the input and the output
 * in the stored order (stream-ordered, counted against the budget). */
SYSTEC_API int systec_tensor_create_csr_ex(int64_t n, int64_t nnz, const int32_t* rowptr,
                                           const int32_t* col, const float* val, int relabel,
                                           systec_stream stream, systec_tensor** out);
SYSTEC_API int systec_tensor_create_coo(int order, int64_t I, int64_t nnz,
                                        const int32_t* const* idx, const float* val,
                                        systec_stream stream, systec_tensor** out);
/* order (2 for a matrix), dim (n or I), stored nnz, effective nnz (entries of
 * the expanded tensor), device bytes held. Any output pointer may be NULL. */
SYSTEC_API int systec_tensor_info(const systec_tensor* t, int* order, int64_t* dim,
                                  int64_t* nnz, int64_t* effective_nnz, uint64_t* bytes);
/* The device bytes a prepared operand holds (what systec_serve_register
 * charges against the budget). Errors: EINVAL (NULL argument). */
SYSTEC_API int systec_tensor_bytes(const systec_tensor* t, uint64_t* bytes);
/* The vertex order a prepared matrix is stored in. *relabeled (may be NULL)
 * is 1 if systec_tensor_create_csr_ex relabeled it, else 0. If perm is not
 * NULL and the matrix was relabeled, perm (device int32[n], caller-owned)
 * receives the order: perm[i] is the caller's vertex stored at position i,
 * written on `stream` (asynchronous). Not a matrix: SYSTEC_EINVAL. */
SYSTEC_API int systec_tensor_vertex_order(const systec_tensor* t, int* relabeled, int32_t* perm,
                                          systec_stream stream);
SYSTEC_API int systec_tensor_destroy(systec_tensor* t);
/* y = A x for a prepared matrix; x, y as for systec_ssymv. */
SYSTEC_API int systec_ssymv_t(const systec_tensor* t, const void* x, systec_dtype xdt, float* y,
                              systec_stream stream);
/* s = x^T A x for a prepared matrix; x and out as for systec_syprd (one
 * FP32 partial per chunk of the prepared format, FP64 final sum). A matrix
 * stored with its vertices relabeled permutes x in first (into the handle's
 * work vector). */
SYSTEC_API int systec_syprd_t(const systec_tensor* t, const void* x, systec_dtype xdt, double* out,
                              systec_stream stream);
/* systec_ssymv_t / systec_syprd_t with the vertex order of x and y chosen
 * by the caller: SYSTEC_ORDER_CALLER (0) is what those calls do;
 * SYSTEC_ORDER_STORED (1) takes x and returns y in the order the matrix is
 * stored in (x_stored[i] = x[perm[i]], perm from systec_tensor_vertex_order)
 * and runs no permutation, for callers such as iterative solvers that keep
 * their vectors in that order between calls. For a matrix that was not
 * relabeled both orders are the caller's. Anything else is SYSTEC_EINVAL. */
enum { SYSTEC_ORDER_CALLER = 0, SYSTEC_ORDER_STORED = 1 };
SYSTEC_API int systec_ssymv_t_ex(const systec_tensor* t, const void* x, systec_dtype xdt, float* y,
                                 int vertex_order, systec_stream stream);
SYSTEC_API int systec_syprd_t_ex(const systec_tensor* t, const void* x, systec_dtype xdt,
                                 double* out, int vertex_order, systec_stream stream);
/* The Bellman-Ford update for a prepared matrix; d and y as for
 * systec_bellman_ford (in the caller's vertex order; a relabeled matrix
 * permutes d in and y out through the handle's work vectors). */
SYSTEC_API int systec_bellman_ford_t(const systec_tensor* t, const float* d, float* y,
                                     systec_stream stream);
/* C = MTTKRP for a prepared tensor; B, C as for systec_mttkrp. */
SYSTEC_API int systec_mttkrp_t(const systec_tensor* t, const void* B, systec_dtype bdt,
                               int64_t R, float* C, systec_stream stream);
/* ------------------------------------------------------------------------
 * One step of symmetric CP-ALS around MTTKRP (Sec. 5.2.6: a symmetric CP
 * decomposition models T by one factor matrix B, T ~ [[B]] = sum_r b_r (x)
 * ... (x) b_r, so the least-squares update is the same in every mode):
 *   C      = MTTKRP(T, B)                  (as systec_mttkrp_t, slot views)
 *   G      = B^T B                         (R x R)
 *   B_new  = C (G^(N-1))^-1                (elementwise power; Cholesky)
 *   fit    = { ||T||^2, <T, [[B]]>, ||[[B]]||^2, ||T - [[B]]||^2 }
 * with ||T||^2 = sum over stored entries of (distinct permutations) v^2,
 * <T,[[B]]> = sum C .* B and ||[[B]]||^2 = sum G.^N.
 *   t       a prepared tensor of order 3..5
 *   B       device I x R row-major, dtype bdt (F32 or BF16); 1 <= R <= 64
 *   C       device float I x R (the MTTKRP), overwritten
 *   B_new   device float I x R, overwritten
 *   G       device float R x R, overwritten
 *   fit     device double[4], overwritten (FP32 partial sums, FP64 final)
 * If G^(N-1) is not positive definite (B without full column rank) B_new
 * is NaN. Stream-ordered workspace of about 2 KiB * R^2 is taken and
 * returned inside the call. Errors: EINVAL, EDEVICE.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_cp_step(const systec_tensor* t, const void* B, systec_dtype bdt,
                              int64_t R, float* C, float* B_new, float* G, double* fit,
                              systec_stream stream);
/* systec_mttkrp_t with an explicit algorithm (systec_mttkrp_t is AUTO: the
 * one-lane-per-entry LDS form where it applies, else the slot views).
 * ATOMIC runs on the tensor's canonical list (its first view). */
SYSTEC_API int systec_mttkrp_t_ex(const systec_tensor* t, const void* B, systec_dtype bdt,
                                  int64_t R, float* C, systec_mttkrp_algo algo,
                                  systec_stream stream);

/* ------------------------------------------------------------------------
 * Serving: many prepared operands resident in HBM, requests of mixed kind
 * and size batched continuously into step launches.
 *
 * A server owns streams on `device` and a scheduler thread. Registered
 * tensors (systec_serve_register takes ownership of a systec_tensor; it is
 * freed by the server) count against budget_bytes while registered. A
 * request names a registered tensor, an input (x for a matrix, B with R
 * columns for a tensor; dtype F32 or BF16) and an output (y or C, FP32) in
 * device memory; their bytes are charged from admission to completion.
 * Requests are admitted in arrival order while fewer than max_slots are
 * running and the bytes fit; a request that could never fit returns
 * SYSTEC_EBUDGET from submit, and more than max_queue waiting requests
 * return SYSTEC_EBUSY. Each step takes work (chunks of the prepared
 * operands, at most step_work_nnz entries in total) from every running
 * request round-robin and runs it as one launch per kernel kind and
 * variant, one workgroup per work unit; a
 * request submitted while a step runs joins the next step. The output is
 * zeroed by the server; it is complete when wait returns SYSTEC_OK or poll
 * reports state 2. Latency is measured from arrival_ns (a time from
 * systec_serve_now_ns; 0 means "now") to completion, so it includes
 * queueing. In and out buffers must stay valid until the request completes
 * or fails. R is limited to 1..64. A failed step marks every request in it
 * failed (state 3; wait returns SYSTEC_EDEVICE with the message).
 * destroy fails queued requests, drains running ones and frees the tensors.
 * ---------------------------------------------------------------------- */
typedef struct systec_server systec_server;
typedef struct {
  uint64_t budget_bytes;  /* resident tensors + in-flight request buffers */
  int32_t max_slots;      /* requests running at once */
  int64_t step_work_nnz;  /* work per step, in stored entries: larger steps raise
                             throughput, smaller steps lower the latency of small
                             requests sharing steps with large ones */
  int32_t device;         /* HIP device ordinal */
  int32_t max_queue;      /* waiting requests before SYSTEC_EBUSY (<= 0: 2^20) */
  int32_t max_inflight;   /* steps queued on the device at once (<= 0: 2; at most 4); a
                             request admitted now starts after the steps
                             already queued, so fewer steps lower latency and
                             one step leaves the device idle between steps */
  int32_t streams;        /* 1: the kernel kinds of a step run one after another on
                             one stream; 0: one stream per kind (SSYMV, MTTKRP of
                             order 3, 4, 5), so that the kinds overlap */
  int64_t min_step_work_nnz; /* work per step with one running request; the step
                                budget grows linearly to step_work_nnz with
                                max_slots running (<= 0: always step_work_nnz) */
} systec_serve_config;
typedef struct {
  int64_t submitted, completed, failed, rejected, steps, queued, running;
  double p50_us, p99_us, mean_us, max_us; /* latency of completed requests */
  double req_per_s, eff_nnz_per_s;        /* from first arrival to last completion */
  uint64_t bytes_in_use;
} systec_serve_stats;

SYSTEC_API int systec_serve_create(const systec_serve_config* cfg, systec_server** out);
SYSTEC_API int systec_serve_register(systec_server* s, systec_tensor* t, int64_t* tensor_id);
SYSTEC_API int systec_serve_unregister(systec_server* s, int64_t tensor_id);
/* The server's streams do not wait for the caller's: `in` must hold its
 * values and `out` must be free of earlier work when systec_serve_submit is
 * called (for example after synchronizing the stream that wrote them).
 * systec_serve_submit_after orders the request after the work enqueued on
 * the caller's stream `after` so far instead: the server's stream waits on
 * the device for that work before it zeroes `out` and reads `in`, and the
 * caller need not synchronize (torch: after = current_stream). */
SYSTEC_API int systec_serve_submit(systec_server* s, int64_t tensor_id, const void* in,
                                   systec_dtype dt, int64_t R, float* out, int64_t arrival_ns,
                                   int64_t* req_id);
SYSTEC_API int systec_serve_submit_after(systec_server* s, int64_t tensor_id, const void* in,
                                         systec_dtype dt, int64_t R, float* out,
                                         int64_t arrival_ns, systec_stream after,
                                         int64_t* req_id);
/* state: 0 queued, 1 running, 2 done, 3 failed */
SYSTEC_API int systec_serve_poll(systec_server* s, int64_t req_id, int* state);
/* timeout_us < 0 waits without limit; SYSTEC_ETIMEOUT when it expires */
SYSTEC_API int systec_serve_wait(systec_server* s, int64_t req_id, int64_t timeout_us);
SYSTEC_API int systec_serve_get_stats(systec_server* s, systec_serve_stats* out);
SYSTEC_API int systec_serve_reset_stats(systec_server* s);
SYSTEC_API int64_t systec_serve_now_ns(void);
SYSTEC_API int systec_serve_destroy(systec_server* s);

/* ------------------------------------------------------------------------
 * Kernel timing. When enabled, the library records a pair of HIP events
 * around every launch of a hot kernel (SSYMV, SYPRD, MTTKRP and the
 * comparison kernels) on the stream it is launched on.
 * systec_kernel_timing_read synchronizes those events and returns the
 * summed duration (milliseconds) and the number of launches timed since the
 * last read, then resets both. Not thread-safe with concurrent launches.
 * ---------------------------------------------------------------------- */
SYSTEC_API int systec_kernel_timing(int enable);
SYSTEC_API int systec_kernel_timing_read(double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* SYSTEC_H */
