// Runs every oracle function on seeded random and degenerate inputs, for a build under
// AddressSanitizer and UndefinedBehaviorSanitizer: any out-of-bounds access, use of freed
// memory, signed overflow or misaligned access aborts the run.  Also checks the invariants
// the two assembly reads share (monotone offsets, strictly increasing rows, equal bits).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

extern "C" {
int oracle_coo_to_csc_rbt(int64_t, int64_t, int64_t, const int32_t*, const int32_t*,
                          const double*, int32_t*, int32_t*, double*, int64_t*);
int oracle_coo_to_csc_sort(int64_t, int64_t, int64_t, const int32_t*, const int32_t*,
                           const double*, int32_t*, int32_t*, double*, int64_t*);
int oracle_csc_insert(int64_t, int64_t, const int32_t*, const int32_t*, const double*, int64_t,
                      const int32_t*, const int32_t*, const double*, int32_t*, int32_t*,
                      double*, int64_t*);
int oracle_csc_add(int64_t, int64_t, const int32_t*, const int32_t*, const double*,
                   const int32_t*, const int32_t*, const double*, int32_t*, int32_t*, double*,
                   int64_t*);
int oracle_csc_transpose(int64_t, int64_t, const int32_t*, const int32_t*, const double*,
                         int32_t*, int32_t*, double*);
int oracle_trace_atb(int64_t, int64_t, const int32_t*, const int32_t*, const double*,
                     const int32_t*, const int32_t*, const double*, double*, int64_t*);
void oracle_triplet_grad(int64_t, int64_t, int64_t, int64_t, const int32_t*, const int32_t*,
                         const double*, const double*, double*, double*);
void oracle_spmm(int64_t, int64_t, int64_t, const int32_t*, const int32_t*, const double*,
                 const double*, double*, double*, int64_t*);
void oracle_spmm_backward(int64_t, int64_t, int64_t, const int32_t*, const int32_t*,
                          const double*, const double*, const double*, double*, double*,
                          double*, double*);
void oracle_column_sums(int64_t, const int32_t*, const double*, double*);
}

namespace {

int g_fail = 0;
void check(bool ok, const char* what, int seed) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s (case %d)\n", what, seed);
    ++g_fail;
  }
}

struct Csc {
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  std::vector<int32_t> cp, ri;
  std::vector<double> v;
};

Csc assemble(int64_t nr, int64_t nc, const std::vector<int32_t>& r, const std::vector<int32_t>& c,
             const std::vector<double>& v, int seed) {
  const int64_t n = (int64_t)r.size();
  Csc a, b;
  for (Csc* x : {&a, &b}) {
    x->n_rows = nr;
    x->n_cols = nc;
    x->cp.assign(nc + 1, -1);
    x->ri.assign(n > 0 ? n : 1, -1);
    x->v.assign(n > 0 ? n : 1, 0.0);
  }
  const int s1 = oracle_coo_to_csc_rbt(nr, nc, n, r.data(), c.data(), v.data(), a.cp.data(),
                                       a.ri.data(), a.v.data(), &a.nnz);
  const int s2 = oracle_coo_to_csc_sort(nr, nc, n, r.data(), c.data(), v.data(), b.cp.data(),
                                        b.ri.data(), b.v.data(), &b.nnz);
  check(s1 == s2, "both assembly reads give one status", seed);
  if (s1 != 0) return a;
  check(a.nnz == b.nnz && a.cp == b.cp, "both reads give one structure", seed);
  for (int64_t p = 0; p < a.nnz; ++p) {
    check(a.ri[p] == b.ri[p], "row indices agree", seed);
    check(std::memcmp(&a.v[p], &b.v[p], sizeof(double)) == 0 || (std::isnan(a.v[p]) &&
                                                                  std::isnan(b.v[p])),
          "values agree bit for bit", seed);
  }
  check(a.cp[0] == 0 && a.cp[nc] == a.nnz, "offsets start at 0, end at nnz", seed);
  for (int64_t j = 0; j < nc; ++j) {
    check(a.cp[j] <= a.cp[j + 1], "offsets monotone", seed);
    for (int64_t p = a.cp[j] + 1; p < a.cp[j + 1]; ++p)
      check(a.ri[p - 1] < a.ri[p], "rows increase down a column", seed);
  }
  return a;
}

void one_case(int seed, int64_t nr, int64_t nc, int64_t n, int64_t k, bool out_of_range) {
  std::mt19937_64 rng(seed);
  std::vector<int32_t> r(n), c(n);
  std::vector<double> v(n);
  for (int64_t t = 0; t < n; ++t) {
    r[t] = nr > 0 ? (int32_t)(rng() % nr) : 0;
    c[t] = nc > 0 ? (int32_t)(rng() % nc) : 0;
    const int pick = (int)(rng() % 8);
    v[t] = pick == 0 ? 0.0 : pick == 1 ? -0.0 : pick == 2 ? 0.5 : pick == 3 ? -0.5
         : (double)(int64_t)(rng() % 2001 - 1000) / 64.0;
  }
  if (n > 3 && seed % 7 == 0) {  // a NaN and an infinity
    v[0] = std::nan("");
    v[1] = INFINITY;
  }
  if (out_of_range && n > 0) r[n / 2] = (int32_t)nr;
  Csc A = assemble(nr, nc, r, c, v, seed);
  if (out_of_range && n > 0) return;
  if (nr == 0 || nc == 0) return;
  // second matrix for insertion, sum and trace
  std::vector<int32_t> r2(n / 2 + 1), c2(n / 2 + 1);
  std::vector<double> v2(n / 2 + 1);
  for (size_t t = 0; t < r2.size(); ++t) {
    r2[t] = (int32_t)(rng() % nr);
    c2[t] = (int32_t)(rng() % nc);
    v2[t] = (double)(int64_t)(rng() % 201 - 100) / 8.0;
  }
  Csc B = assemble(nr, nc, r2, c2, v2, seed + 1000);
  const int64_t cap = A.nnz + (int64_t)r2.size();
  std::vector<int32_t> cp(nc + 1), ri(cap > 0 ? cap : 1);
  std::vector<double> vo(cap > 0 ? cap : 1);
  int64_t nnz = 0;
  check(oracle_csc_insert(nr, nc, A.cp.data(), A.ri.data(), A.v.data(), (int64_t)r2.size(),
                          r2.data(), c2.data(), v2.data(), cp.data(), ri.data(), vo.data(),
                          &nnz) == 0, "insert", seed);
  const int64_t cap2 = A.nnz + B.nnz;
  std::vector<int32_t> cps(nc + 1), ris(cap2 > 0 ? cap2 : 1);
  std::vector<double> vs(cap2 > 0 ? cap2 : 1);
  check(oracle_csc_add(nr, nc, A.cp.data(), A.ri.data(), A.v.data(), B.cp.data(), B.ri.data(),
                       B.v.data(), cps.data(), ris.data(), vs.data(), &nnz) == 0, "add", seed);
  std::vector<int32_t> tcp(nr + 1), tri(A.nnz > 0 ? A.nnz : 1);
  std::vector<double> tv(A.nnz > 0 ? A.nnz : 1);
  check(oracle_csc_transpose(nr, nc, A.cp.data(), A.ri.data(), A.v.data(), tcp.data(),
                             tri.data(), tv.data()) == 0, "transpose", seed);
  double tr = 0.0;
  int64_t hits = 0;
  check(oracle_trace_atb(nr, nc, A.cp.data(), A.ri.data(), A.v.data(), B.cp.data(),
                         B.ri.data(), B.v.data(), &tr, &hits) == 0, "trace", seed);
  std::vector<double> X(nc * k), G(nr * k), Y(nr * k), S(nr * k), dX(nc * k), SdX(nc * k);
  std::vector<double> dval(A.nnz > 0 ? A.nnz : 1), Sdv(A.nnz > 0 ? A.nnz : 1);
  std::vector<int64_t> M(nr);
  for (auto& x : X) x = (double)(int64_t)(rng() % 17 - 8) / 4.0;
  for (auto& x : G) x = (double)(int64_t)(rng() % 17 - 8) / 4.0;
  oracle_spmm(nr, nc, k, A.cp.data(), A.ri.data(), A.v.data(), X.data(), Y.data(), S.data(),
              M.data());
  oracle_spmm_backward(nr, nc, k, A.cp.data(), A.ri.data(), A.v.data(), G.data(), X.data(),
                       dX.data(), dval.data(), SdX.data(), Sdv.data());
  std::vector<double> dv(n > 0 ? n : 1), St(n > 0 ? n : 1), cs(nc);
  oracle_triplet_grad(nr, nc, n, k, r.data(), c.data(), G.data(), X.data(), dv.data(),
                      St.data());
  oracle_column_sums(nc, A.cp.data(), A.v.data(), cs.data());
}

}  // namespace

int main() {
  int seed = 1;
  const int64_t shapes[][2] = {{1, 1}, {1, 9}, {9, 1}, {7, 3}, {64, 64}, {300, 40}, {40, 300}};
  for (const auto& sh : shapes)
    for (int64_t n : {0, 1, 5, 200, 3000})
      for (int64_t k : {1, 3, 8}) {
        one_case(seed++, sh[0], sh[1], n, k, false);
        if (n > 0) one_case(seed++, sh[0], sh[1], n, k, true);
      }
  one_case(seed++, 0, 5, 0, 2, false);
  one_case(seed++, 5, 0, 0, 2, false);
  // invalid arguments are reported, never dereferenced
  int64_t nnz = 0;
  int32_t cp[2] = {0, 0};
  check(oracle_coo_to_csc_sort(-1, 1, 0, nullptr, nullptr, nullptr, cp, nullptr, nullptr,
                               &nnz) == 1, "negative size", 0);
  check(oracle_coo_to_csc_rbt(1, 1, 3, nullptr, nullptr, nullptr, cp, nullptr, nullptr,
                              &nnz) == 1, "null arrays", 0);
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("oracle driver: %d cases clean\n", seed - 1);
  return 0;
}
