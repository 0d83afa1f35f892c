// spm oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, deliberately unoptimised CPU reference for what the sparse path computes:
// bulk assembly of coordinate (COO) triplets into compressed sparse column (CSC) form, the CSC
// sparse x dense product Y = A.X, and its adjoint (dX = A^T.G, dvalues = G.X sampled on A's
// pattern); batch insertion into an existing CSC, the sum of two CSCs, the transpose,
// trace(A^T B), and the gradient with respect to each input triplet.  Everything is IEEE binary64; the build uses -O2 -ffp-contract=off and no fast-math,
// so every '+' and '*' below is one correctly rounded binary64 operation, in the order written.
//
// Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may load this
// library.  It shares no code, header, table or helper with the GPU implementation.
//
// Paper: C. Sanderson, R. Curtin, "A User-Friendly Hybrid Sparse Matrix Class in C++", LNCS 10931
// (2018), arXiv:1805.03380.
//
// Status codes returned here match the public ones by value only (0 ok, 1 invalid argument,
// 2 triplet out of range); the numbers are retyped, not shared.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>
#include <algorithm>
#include <climits>

namespace {

// Section 3.1: zero-based row / column indices; a triplet whose location lies outside the
// n_rows x n_cols matrix has no place in the CSC arrays and is rejected.
bool in_range(int64_t n_rows, int64_t n_cols, int32_t r, int32_t c) {
  return r >= 0 && c >= 0 && (int64_t)r < n_rows && (int64_t)c < n_cols;
}

// Section 3.1: column offsets.  c[0] = 0, c[n_cols] = N, and column i holds c[i+1] - c[i]
// elements.  Built from the column of each emitted element, in emission order.
void offsets_from_columns(int64_t n_cols, const std::vector<int64_t>& emitted_cols,
                          int32_t* col_ptr) {
  std::vector<int64_t> count(n_cols + 1, 0);
  for (int64_t c : emitted_cols) count[c + 1] += 1;
  col_ptr[0] = 0;
  for (int64_t i = 0; i < n_cols; ++i) col_ptr[i + 1] = (int32_t)(col_ptr[i] + count[i + 1]);
}

// A CSC whose offsets start at 0 and never decrease, and whose stored rows lie in the matrix and
// strictly increase down each column (Section 3.1: each column lists its rows in order).
bool valid_sorted_csc(int64_t n_rows, int64_t n_cols, const int32_t* col_ptr,
                      const int32_t* row_idx) {
  if (!col_ptr || col_ptr[0] != 0) return false;
  for (int64_t c = 0; c < n_cols; ++c) {
    if (col_ptr[c + 1] < col_ptr[c]) return false;
    for (int64_t p = col_ptr[c]; p < col_ptr[c + 1]; ++p) {
      if (row_idx[p] < 0 || (int64_t)row_idx[p] >= n_rows) return false;
      if (p > col_ptr[c] && row_idx[p] <= row_idx[p - 1]) return false;
    }
  }
  return true;
}

}  // namespace

extern "C" {

// Assembly, read 1 (the paper's own route, Section 3.3 and Section 3.4):
//   every triplet is an element insertion into a red-black tree (std::map is one) keyed by the
//   location index  index = row + column * n_rows  (column-major encoding, Section 3.3);
//   repeated locations accumulate, like X(r,c) += v in Fig. 1, in input order;
//   the sync to CSC is an in-order traversal (smallest to largest index == column-major order),
//   decoding row = index mod n_rows and column = floor(index / n_rows).
// Exact zeros are not stored: a location whose accumulated value compares equal to 0.0 (this
// includes -0.0 and cancelled sums) is skipped during the traversal.  NaN and Inf are stored.
// Output arrays: col_ptr[n_cols+1]; row_idx and val_out have capacity nnz_in.
// Returns 0, 1 (bad sizes / null pointers) or 2 (some triplet out of range; outputs untouched).
int oracle_coo_to_csc_rbt(int64_t n_rows, int64_t n_cols, int64_t nnz_in, const int32_t* row,
                          const int32_t* col, const double* val, int32_t* col_ptr,
                          int32_t* row_idx, double* val_out, int64_t* nnz_out) {
  if (n_rows < 0 || n_cols < 0 || nnz_in < 0 || !col_ptr || !nnz_out) return 1;
  if (nnz_in > 0 && (!row || !col || !val || !row_idx || !val_out)) return 1;
  for (int64_t t = 0; t < nnz_in; ++t)
    if (!in_range(n_rows, n_cols, row[t], col[t])) return 2;

  std::map<uint64_t, double> tree;  // a red-black tree of (index, value)
  for (int64_t t = 0; t < nnz_in; ++t) {
    uint64_t index = (uint64_t)row[t] + (uint64_t)col[t] * (uint64_t)n_rows;
    auto it = tree.find(index);
    if (it == tree.end())
      tree.emplace(index, val[t]);
    else
      it->second = it->second + val[t];
  }

  std::vector<int64_t> emitted_cols;
  int64_t n = 0;
  for (const auto& kv : tree) {
    if (kv.second == 0.0) continue;  // exact zero: not stored
    int64_t r = (int64_t)(kv.first % (uint64_t)n_rows);
    int64_t c = (int64_t)(kv.first / (uint64_t)n_rows);
    row_idx[n] = (int32_t)r;
    val_out[n] = kv.second;
    emitted_cols.push_back(c);
    ++n;
  }
  offsets_from_columns(n_cols, emitted_cols, col_ptr);
  *nnz_out = n;
  return 0;
}

// Assembly, read 2 (batch form of the same definition, Section 3.1 "sort, then merge"):
//   stable sort of the triplets by (column, row) -- column-major order -- so that triplets at
//   one location stay in input order; then each run of equal locations is folded left to right,
//   s = ((v_t1 + v_t2) + v_t3) + ...; the location is stored iff s != 0.0.
// Same contract and outputs as oracle_coo_to_csc_rbt; the two must agree bit for bit.
int oracle_coo_to_csc_sort(int64_t n_rows, int64_t n_cols, int64_t nnz_in, const int32_t* row,
                           const int32_t* col, const double* val, int32_t* col_ptr,
                           int32_t* row_idx, double* val_out, int64_t* nnz_out) {
  if (n_rows < 0 || n_cols < 0 || nnz_in < 0 || !col_ptr || !nnz_out) return 1;
  if (nnz_in > 0 && (!row || !col || !val || !row_idx || !val_out)) return 1;
  for (int64_t t = 0; t < nnz_in; ++t)
    if (!in_range(n_rows, n_cols, row[t], col[t])) return 2;

  std::vector<int64_t> order(nnz_in);
  for (int64_t t = 0; t < nnz_in; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    if (col[a] != col[b]) return col[a] < col[b];
    return row[a] < row[b];
  });

  std::vector<int64_t> emitted_cols;
  int64_t n = 0;
  int64_t i = 0;
  while (i < nnz_in) {
    int64_t j = i;
    double s = val[order[i]];
    ++j;
    while (j < nnz_in && col[order[j]] == col[order[i]] && row[order[j]] == row[order[i]]) {
      s = s + val[order[j]];
      ++j;
    }
    if (s != 0.0) {
      row_idx[n] = row[order[i]];
      val_out[n] = s;
      emitted_cols.push_back(col[order[i]]);
      ++n;
    }
    i = j;
  }
  offsets_from_columns(n_cols, emitted_cols, col_ptr);
  *nnz_out = n;
  return 0;
}

// Batch insertion into an existing CSC (Section 3.1: sort the elements to be inserted, then
// merge them with the existing arrays), with the accumulating update of Fig. 1, X(r,c) += v:
//   the new triplets are stably sorted by (column, row), so that those at one location stay in
//   input order; every column of the result is the merge of the existing column (rows
//   strictly increasing) with the sorted new triplets of that column; at each location the
//   existing value, if any, comes first and the new values are added to it left to right in
//   binary64, s = ((a + v_t1) + v_t2) + ... (a location without an existing element starts
//   from its first new value); the location is stored iff s != 0.0.
// Existing CSC: a_col_ptr[n_cols+1] with a_col_ptr[0] = 0 and non-decreasing offsets, and
// a_row_idx / a_val holding a_col_ptr[n_cols] elements.  Outputs as for assembly, with
// capacity a_col_ptr[n_cols] + nnz_in.
// Returns 0, 1 (bad sizes, null pointers, or an existing CSC not of that form) or 2 (a new
// triplet out of range; outputs untouched).
int oracle_csc_insert(int64_t n_rows, int64_t n_cols, const int32_t* a_col_ptr,
                      const int32_t* a_row_idx, const double* a_val, int64_t nnz_in,
                      const int32_t* row, const int32_t* col, const double* val,
                      int32_t* col_ptr, int32_t* row_idx, double* val_out, int64_t* nnz_out) {
  if (n_rows < 0 || n_cols < 0 || nnz_in < 0 || !a_col_ptr || !col_ptr || !nnz_out) return 1;
  if (nnz_in > 0 && (!row || !col || !val)) return 1;
  if (a_col_ptr[0] != 0) return 1;
  for (int64_t c = 0; c < n_cols; ++c) {
    if (a_col_ptr[c + 1] < a_col_ptr[c]) return 1;
    for (int64_t p = a_col_ptr[c]; p < a_col_ptr[c + 1]; ++p) {
      if (a_row_idx[p] < 0 || (int64_t)a_row_idx[p] >= n_rows) return 1;
      if (p > a_col_ptr[c] && a_row_idx[p] <= a_row_idx[p - 1]) return 1;
    }
  }
  for (int64_t t = 0; t < nnz_in; ++t)
    if (!in_range(n_rows, n_cols, row[t], col[t])) return 2;

  std::vector<int64_t> order(nnz_in);
  for (int64_t t = 0; t < nnz_in; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return col[a] < col[b] || (col[a] == col[b] && row[a] < row[b]);
  });

  std::vector<int64_t> emitted_cols;
  int64_t n = 0;
  int64_t j = 0;  // next sorted new triplet
  for (int64_t c = 0; c < n_cols; ++c) {
    int64_t p = a_col_ptr[c];
    const int64_t pe = a_col_ptr[c + 1];
    while (p < pe || (j < nnz_in && col[order[j]] == c)) {
      // the next location of the merged column: the smaller of the two next rows
      int64_t r = p < pe ? a_row_idx[p] : INT64_MAX;
      if (j < nnz_in && col[order[j]] == c && row[order[j]] < r) r = row[order[j]];
      bool started = false;
      double acc = 0.0;
      if (p < pe && a_row_idx[p] == r) {  // the existing element first
        acc = a_val[p];
        started = true;
        ++p;
      }
      while (j < nnz_in && col[order[j]] == c && row[order[j]] == r) {
        acc = started ? acc + val[order[j]] : val[order[j]];
        started = true;
        ++j;
      }
      if (acc != 0.0) {
        row_idx[n] = (int32_t)r;
        val_out[n] = acc;
        emitted_cols.push_back(c);
        ++n;
      }
    }
  }
  offsets_from_columns(n_cols, emitted_cols, col_ptr);
  *nnz_out = n;
  return 0;
}

// Sparse sum A + B of two CSCs of one shape (the addition of two sparse matrices, built, like
// batch insertion, by merging sorted columns; Section 3.1).  Column by column, the two sorted
// row lists are merged: a row stored in both gives A's value plus B's value (binary64, A's
// first), a row stored in one gives that value; a result equal to 0.0 is not stored (the rule
// of the assembly).  Output capacity: nnz(A) + nnz(B).
// Returns 0, or 1 (bad sizes, null pointers, or a CSC that is not valid and sorted).
int oracle_csc_add(int64_t n_rows, int64_t n_cols, const int32_t* a_col_ptr,
                   const int32_t* a_row_idx, const double* a_val, const int32_t* b_col_ptr,
                   const int32_t* b_row_idx, const double* b_val, int32_t* col_ptr,
                   int32_t* row_idx, double* val_out, int64_t* nnz_out) {
  if (n_rows < 0 || n_cols < 0 || !col_ptr || !nnz_out) return 1;
  if (!valid_sorted_csc(n_rows, n_cols, a_col_ptr, a_row_idx)) return 1;
  if (!valid_sorted_csc(n_rows, n_cols, b_col_ptr, b_row_idx)) return 1;
  int64_t n = 0;
  col_ptr[0] = 0;
  for (int64_t c = 0; c < n_cols; ++c) {
    int64_t p = a_col_ptr[c], q = b_col_ptr[c];
    const int64_t pe = a_col_ptr[c + 1], qe = b_col_ptr[c + 1];
    while (p < pe || q < qe) {
      int32_t r;
      double v;
      if (q >= qe || (p < pe && a_row_idx[p] < b_row_idx[q])) {
        r = a_row_idx[p];
        v = a_val[p];
        ++p;
      } else if (p >= pe || b_row_idx[q] < a_row_idx[p]) {
        r = b_row_idx[q];
        v = b_val[q];
        ++q;
      } else {  // the row is stored in both
        r = a_row_idx[p];
        v = a_val[p] + b_val[q];
        ++p;
        ++q;
      }
      if (v != 0.0) {
        row_idx[n] = r;
        val_out[n] = v;
        ++n;
      }
    }
    col_ptr[c + 1] = (int32_t)n;
  }
  *nnz_out = n;
  return 0;
}

// Transpose X.t() (Table 1) of a CSC, written as a CSC of the n_cols x n_rows result:
//   every stored element (r, c, v) of A becomes (c, r, v) of A^T.  Column r of A^T lists the
//   elements of row r of A in increasing column order (a counting pass over the rows of A,
//   then the columns of A walked in order, so each row receives its elements by increasing
//   column).  Values are moved, not changed.
// Output: t_col_ptr[n_rows+1], t_row_idx / t_val with capacity a_col_ptr[n_cols].
// Returns 0, or 1 (bad sizes, null pointers, or an existing CSC that is not valid).
int oracle_csc_transpose(int64_t n_rows, int64_t n_cols, const int32_t* a_col_ptr,
                         const int32_t* a_row_idx, const double* a_val, int32_t* t_col_ptr,
                         int32_t* t_row_idx, double* t_val) {
  if (n_rows < 0 || n_cols < 0 || !a_col_ptr || !t_col_ptr) return 1;
  if (a_col_ptr[0] != 0) return 1;
  for (int64_t c = 0; c < n_cols; ++c) {
    if (a_col_ptr[c + 1] < a_col_ptr[c]) return 1;
    for (int64_t p = a_col_ptr[c]; p < a_col_ptr[c + 1]; ++p)
      if (a_row_idx[p] < 0 || (int64_t)a_row_idx[p] >= n_rows) return 1;
  }
  std::vector<int64_t> per_row(n_rows + 1, 0);
  for (int64_t p = 0; p < a_col_ptr[n_cols]; ++p) per_row[a_row_idx[p] + 1] += 1;
  t_col_ptr[0] = 0;
  for (int64_t r = 0; r < n_rows; ++r) t_col_ptr[r + 1] = (int32_t)(t_col_ptr[r] + per_row[r + 1]);
  std::vector<int64_t> next(n_rows);
  for (int64_t r = 0; r < n_rows; ++r) next[r] = t_col_ptr[r];
  for (int64_t c = 0; c < n_cols; ++c)
    for (int64_t p = a_col_ptr[c]; p < a_col_ptr[c + 1]; ++p) {
      const int64_t q = next[a_row_idx[p]]++;
      t_row_idx[q] = (int32_t)c;
      t_val[q] = a_val[p];
    }
  return 0;
}

// trace(A^T B) (Section 2's example of an expression evaluated without forming the transpose
// or the product; Table 1).  Entry (j, j) of A^T B is the dot product of column j of A with
// column j of B, so the trace is the sum, over every location stored in both A and B, of
// A[i,j] * B[i,j].  A location stored in only one of them meets a structural zero and adds
// nothing.  Columns are taken in ascending order and, within a column, A's stored rows in
// ascending order; B's element at the same row is found by binary search in B's sorted
// column.  Each product is one binary64 multiply, and the products are added left to right.
// Outputs: *out = the trace, *hits = the number of locations stored in both.
// Returns 0, or 1 (bad sizes, null pointers, or a CSC that is not valid and sorted).
int oracle_trace_atb(int64_t n_rows, int64_t n_cols, const int32_t* a_col_ptr,
                     const int32_t* a_row_idx, const double* a_val, const int32_t* b_col_ptr,
                     const int32_t* b_row_idx, const double* b_val, double* out,
                     int64_t* hits) {
  if (n_rows < 0 || n_cols < 0 || !out || !hits) return 1;
  if (!valid_sorted_csc(n_rows, n_cols, a_col_ptr, a_row_idx)) return 1;
  if (!valid_sorted_csc(n_rows, n_cols, b_col_ptr, b_row_idx)) return 1;
  double trace = 0.0;
  int64_t matched = 0;
  for (int64_t c = 0; c < n_cols; ++c) {
    const int32_t* b_first = b_row_idx + b_col_ptr[c];
    const int32_t* b_last = b_row_idx + b_col_ptr[c + 1];
    for (int64_t p = a_col_ptr[c]; p < a_col_ptr[c + 1]; ++p) {
      const int32_t r = a_row_idx[p];
      const int32_t* it = std::lower_bound(b_first, b_last, r);
      if (it == b_last || *it != r) continue;  // B has no element at (r, c)
      const int64_t q = it - b_row_idx;
      trace = trace + a_val[p] * b_val[q];
      matched += 1;
    }
  }
  *out = trace;
  *hits = matched;
  return 0;
}

// Gradient with respect to each input triplet's value (the triplet-level adjoint of assembly
// followed by Y = A.X, for a loss with dL/dY = G).  Assembly makes A[r,c] the sum of the values
// of the triplets at (r, c) (Fig. 1's +=; a zero sum is merely not stored, the entry is still
// that sum), and L depends on A[r,c] through sum_j G[r,j] A[r,c] X[c,j]; so every triplet t
// at (r, c) has dL/dv_t = sum_j G[r,j] * X[c,j], whether or not its location survived, and
// duplicates share it.  A triplet outside the matrix takes no part in A: its gradient is 0.
// One binary64 multiply per term, added left to right in ascending j; S[t] = sum |G||X|.
void oracle_triplet_grad(int64_t n_rows, int64_t n_cols, int64_t nnz_in, int64_t k,
                         const int32_t* row, const int32_t* col, const double* G,
                         const double* X, double* dv, double* S) {
  for (int64_t t = 0; t < nnz_in; ++t) {
    dv[t] = 0.0;
    S[t] = 0.0;
    if (!in_range(n_rows, n_cols, row[t], col[t])) continue;
    const double* g = G + (int64_t)row[t] * k;
    const double* x = X + (int64_t)col[t] * k;
    double d = 0.0, a = 0.0;
    for (int64_t j = 0; j < k; ++j) {
      d = d + g[j] * x[j];
      a = a + std::fabs(g[j]) * std::fabs(x[j]);
    }
    dv[t] = d;
    S[t] = a;
  }
}

// Sparse x dense product, Section 3 use case (iv) and the CSC traversal of Section 3.1:
//   Y[r, j] = sum over stored (r, c) of  v * X[c, j],   X is n_cols x k, Y is n_rows x k,
// both dense row-major.  The loop walks columns in ascending order and, within a column, the
// stored elements in CSC order; each output therefore accumulates its terms in ascending
// column order, starting from 0.0.
// Alongside each output it accumulates the error scale S[r, j] = sum |v| * |X[c, j]| and the
// number of terms M[r] (the length of row r); a fixed-order binary64 sum of M terms is within
// gamma_M * S of the exact value (Higham, Accuracy and Stability of Numerical Algorithms, 3.1).
void oracle_spmm(int64_t n_rows, int64_t n_cols, int64_t k, const int32_t* col_ptr,
                 const int32_t* row_idx, const double* val, const double* X, double* Y,
                 double* S, int64_t* M) {
  for (int64_t i = 0; i < n_rows * k; ++i) { Y[i] = 0.0; S[i] = 0.0; }
  for (int64_t r = 0; r < n_rows; ++r) M[r] = 0;
  for (int64_t c = 0; c < n_cols; ++c) {
    for (int64_t p = col_ptr[c]; p < col_ptr[c + 1]; ++p) {
      int64_t r = row_idx[p];
      double v = val[p];
      for (int64_t j = 0; j < k; ++j) {
        Y[r * k + j] = Y[r * k + j] + v * X[c * k + j];
        S[r * k + j] = S[r * k + j] + std::fabs(v) * std::fabs(X[c * k + j]);
      }
      M[r] += 1;
    }
  }
}

// Adjoint of Y = A.X for the loss L = sum(Y * G), i.e. dL/dY = G:
//   dX[c, j]   = sum over stored (r, c) of v * G[r, j]        (A^T . G: a walk down column c,
//                 the same traversal as the row-vector times CSC product of Fig. 1)
//   dval[p]    = sum_j G[r_p, j] * X[c_p, j]                   (dense.dense product sampled at
//                 the stored location p of A)
// dX accumulates in CSC order within each column, dval in ascending j.  SdX / Sdv are the
// matching error scales (sum of |terms|); the term counts are the column length for dX and k
// for dval, so they are not returned.
void oracle_spmm_backward(int64_t n_rows, int64_t n_cols, int64_t k, const int32_t* col_ptr,
                          const int32_t* row_idx, const double* val, const double* G,
                          const double* X, double* dX, double* dval, double* SdX, double* Sdv) {
  (void)n_rows;
  for (int64_t c = 0; c < n_cols; ++c) {
    for (int64_t j = 0; j < k; ++j) { dX[c * k + j] = 0.0; SdX[c * k + j] = 0.0; }
    for (int64_t p = col_ptr[c]; p < col_ptr[c + 1]; ++p) {
      int64_t r = row_idx[p];
      double v = val[p];
      double d = 0.0, sd = 0.0;
      for (int64_t j = 0; j < k; ++j) {
        dX[c * k + j] = dX[c * k + j] + v * G[r * k + j];
        SdX[c * k + j] = SdX[c * k + j] + std::fabs(v) * std::fabs(G[r * k + j]);
        d = d + G[r * k + j] * X[c * k + j];
        sd = sd + std::fabs(G[r * k + j]) * std::fabs(X[c * k + j]);
      }
      dval[p] = d;
      Sdv[p] = sd;
    }
  }
}

// Row sums through the CSC arrays, for the sum(X, dim) special case of Table 1.
void oracle_column_sums(int64_t n_cols, const int32_t* col_ptr, const double* val, double* out) {
  for (int64_t c = 0; c < n_cols; ++c) {
    double s = 0.0;
    for (int64_t p = col_ptr[c]; p < col_ptr[c + 1]; ++p) s = s + val[p];
    out[c] = s;
  }
}

}  // extern "C"
