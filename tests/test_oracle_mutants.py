"""Planted mistakes in copies of the oracle (on the CPU) must each fail at least one pin.

Each mutant is the oracle source with one plausible slip -- a dropped or sign-flipped term, a
wrong or swapped index, a transposed operand, a wrong ordering or a skipped rule -- compiled to
a temporary library and swapped in for the real one while the pins run.  All mutations keep
every memory access in bounds.
"""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
import pins

# the existing value of a location folded last instead of first
INSERT_FOLD = """      if (p < pe && a_row_idx[p] == r) {  // the existing element first
        acc = a_val[p];
        started = true;
        ++p;
      }
      while (j < nnz_in && col[order[j]] == c && row[order[j]] == r) {
        acc = started ? acc + val[order[j]] : val[order[j]];
        started = true;
        ++j;
      }
"""
INSERT_FOLD_NEW_FIRST = """      while (j < nnz_in && col[order[j]] == c && row[order[j]] == r) {
        acc = started ? acc + val[order[j]] : val[order[j]];
        started = true;
        ++j;
      }
      if (p < pe && a_row_idx[p] == r) {
        acc = started ? acc + a_val[p] : a_val[p];
        started = true;
        ++p;
      }
"""

MUTANTS = {
    "fold_sign_sort": ("s = s + val[order[j]];", "s = s - val[order[j]];"),
    "fold_last_wins_rbt": ("it->second = it->second + val[t];", "it->second = val[t];"),
    "keep_zero_sort": ("if (s != 0.0) {", "if (true) {"),
    "keep_zero_rbt": ("if (kv.second == 0.0) continue;", ""),
    "row_order_reversed": ("return row[a] < row[b];", "return row[a] > row[b];"),
    "decode_swapped": ("int64_t r = (int64_t)(kv.first % (uint64_t)n_rows);",
                       "int64_t r = (int64_t)(kv.first / (uint64_t)n_rows) % n_rows;"),
    "offsets_shifted": ("for (int64_t c : emitted_cols) count[c + 1] += 1;",
                        "for (int64_t c : emitted_cols) count[c] += 1;"),
    "spmm_wrong_j": ("Y[r * k + j] = Y[r * k + j] + v * X[c * k + j];",
                     "Y[r * k + j] = Y[r * k + j] + v * X[c * k + (k - 1 - j)];"),
    "spmm_sign": ("Y[r * k + j] = Y[r * k + j] + v * X[c * k + j];",
                  "Y[r * k + j] = Y[r * k + j] - v * X[c * k + j];"),
    "spmm_count": ("M[r] += 1;", "M[r] += 2;"),
    "dx_wrong_operand": ("dX[c * k + j] = dX[c * k + j] + v * G[r * k + j];",
                         "dX[c * k + j] = dX[c * k + j] + v * X[c * k + j];"),
    "dval_sign": ("d = d + G[r * k + j] * X[c * k + j];", "d = d - G[r * k + j] * X[c * k + j];"),
    "dval_dropped_term": ("d = d + G[r * k + j] * X[c * k + j];",
                          "if (j) d = d + G[r * k + j] * X[c * k + j];"),
    "insert_existing_ignored": ("acc = a_val[p];", "acc = 0.0;"),
    "insert_keep_zero": ("if (acc != 0.0) {", "if (true) {"),
    "insert_new_first": (INSERT_FOLD, INSERT_FOLD_NEW_FIRST),
    "transpose_index_kept": ("t_row_idx[q] = (int32_t)c;",
                             "t_row_idx[q] = (int32_t)a_row_idx[p];"),
    "transpose_value_from_wrong_slot": ("t_val[q] = a_val[p];", "t_val[q] = a_val[q];"),
    "trace_last_row_skipped": ("""    for (int64_t p = a_col_ptr[c]; p < a_col_ptr[c + 1]; ++p) {
      const int32_t r = a_row_idx[p];""", """    for (int64_t p = a_col_ptr[c]; p + 1 < a_col_ptr[c + 1]; ++p) {
      const int32_t r = a_row_idx[p];"""),
    "trace_match_unchecked": ("if (it == b_last || *it != r) continue;",
                              "if (it == b_last) continue;"),
    "trace_search_all_columns": ("std::lower_bound(b_first, b_last, r);",
                                 "std::lower_bound(b_row_idx, b_row_idx + b_col_ptr[n_cols], r);"),
    "trace_b_value_replaced": ("trace = trace + a_val[p] * b_val[q];",
                               "trace = trace + a_val[p] * a_val[p];"),
    "tgrad_last_term_dropped": ("""    for (int64_t j = 0; j < k; ++j) {
      d = d + g[j] * x[j];""", """    for (int64_t j = 0; j + 1 < k; ++j) {
      d = d + g[j] * x[j];"""),
    "tgrad_wrong_operand": ("d = d + g[j] * x[j];", "d = d + g[j] * g[j];"),
    "tgrad_sign": ("dv[t] = d;", "dv[t] = -d;"),
    "add_b_dropped_when_shared": ("v = a_val[p] + b_val[q];", "v = a_val[p];"),
    "add_keep_zero": ("""      if (v != 0.0) {
        row_idx[n] = r;""", """      if (true) {
        row_idx[n] = r;"""),
}


@pytest.fixture(scope="module")
def source():
    with open(oracle._SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, "mutation site must be unique: %r" % old
    src = tmp_path / "mutant.cpp"
    src.write_text(source.replace(old, new))
    so = tmp_path / ("lib_%s.so" % name)
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", str(src),
                    "-o", str(so)], check=True)
    saved = oracle._load()
    oracle._lib = oracle.configure(ctypes.CDLL(str(so)))
    caught = []
    try:
        for pin in pins.ALL_PINS:
            try:
                pin()
            except AssertionError:
                caught.append(pin.__name__)
                break
    finally:
        oracle._lib = saved
    assert caught, "planted mistake %s passed every pin" % name
