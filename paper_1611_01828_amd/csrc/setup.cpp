// Once-per-problem host work: input validation, the chordal pattern E', the
// selectors H_k (Section 3.1), and the data step 1 caches before iterating
// (Sections 4.2-4.3).
//
// Step 1 eliminates down to the matrix of eq. (FactorizationMatrix),
// F = I + D/2 + A^T A with D = H^T H diagonal.  F is "diagonal plus low
// rank", so the matrix inversion lemma leaves only the m x m matrix
// K = I + A P^{-1} A^T (P = I + D/2) to factorise; it is SPD with eigenvalues
// >= 1.  K is factorised here once (dense Cholesky, or a sparse Cholesky in a
// minimum-degree order when K is sparse) and its triangular factor is what
// the GPU iteration solves with.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <set>

#include "plan.h"

namespace cdcs {

namespace {

const double kSqrt2 = 1.4142135623730951;

int fail(Error& err, int code, const std::string& msg) {
  err.code = code;
  err.msg = msg;
  return code;
}

inline bool finite(double v) { return std::isfinite(v); }

// forward/backward substitution with a dense column-major lower factor
void dense_solve(int32_t m, const std::vector<double>& L, std::vector<double>& g) {
  for (int32_t j = 0; j < m; ++j) {
    double yj = g[j] / L[(size_t)j * m + j];
    g[j] = yj;
    for (int32_t i = j + 1; i < m; ++i) g[i] -= L[(size_t)j * m + i] * yj;
  }
  for (int32_t j = m - 1; j >= 0; --j) {
    double s = g[j];
    for (int32_t i = j + 1; i < m; ++i) s -= L[(size_t)j * m + i] * g[i];
    g[j] = s / L[(size_t)j * m + j];
  }
}

// minimum-degree elimination on an undirected graph; returns the order and,
// per eliminated vertex, its neighbours eliminated later (= the column
// structure of the Cholesky factor in that order).
void min_degree(int32_t m, std::vector<std::set<int32_t>> adj, std::vector<int32_t>& order,
                std::vector<std::vector<int32_t>>& higher) {
  std::vector<char> done(m, 0);
  std::set<std::pair<int32_t, int32_t>> pq;
  for (int32_t v = 0; v < m; ++v) pq.insert({(int32_t)adj[v].size(), v});
  order.clear();
  higher.assign(m, {});
  while (!pq.empty()) {
    auto it = pq.begin();
    int32_t v = it->second;
    pq.erase(it);
    done[v] = 1;
    order.push_back(v);
    std::vector<int32_t> nb(adj[v].begin(), adj[v].end());
    higher[v] = nb;
    for (int32_t u : nb) {
      pq.erase({(int32_t)adj[u].size(), u});
      adj[u].erase(v);
      for (int32_t w : nb)
        if (w != u) adj[u].insert(w);
      pq.insert({(int32_t)adj[u].size(), u});
    }
    adj[v].clear();
  }
}

}  // namespace

void Factor::solve(std::vector<double>& g) const {
  if (dense) {
    dense_solve(m, Ld, g);
    return;
  }
  std::vector<double> z(m);
  for (int32_t i = 0; i < m; ++i) z[i] = g[perm[i]];
  for (int32_t i = 0; i < m; ++i) {
    double s = z[i];
    for (int32_t q = lptr[i]; q < lptr[i + 1]; ++q) s -= lval[q] * z[lcol[q]];
    z[i] = s / diag[i];
  }
  for (int32_t i = m - 1; i >= 0; --i) {
    double s = z[i];
    for (int32_t q = uptr[i]; q < uptr[i + 1]; ++q) s -= uval[q] * z[ucol[q]];
    z[i] = s / diag[i];
  }
  for (int32_t i = 0; i < m; ++i) g[perm[i]] = z[i];
}

int factor_K(int32_t m, const std::vector<int32_t>& aptr, const std::vector<int32_t>& acol,
             const std::vector<double>& aval, const std::vector<double>& pinv, Factor& f,
             Error& err, double shift) {
  f = Factor();
  f.m = m;
  const int64_t nE = (int64_t)pinv.size();
  // columns of A (entry -> constraint rows, ascending)
  std::vector<int64_t> cptr(nE + 1, 0);
  for (int32_t i = 0; i < m; ++i)
    for (int32_t q = aptr[i]; q < aptr[i + 1]; ++q) cptr[acol[q] + 1]++;
  for (int64_t e = 0; e < nE; ++e) cptr[e + 1] += cptr[e];
  std::vector<int32_t> crow(cptr[nE]);
  std::vector<double> cval(cptr[nE]);
  {
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int32_t i = 0; i < m; ++i)
      for (int32_t q = aptr[i]; q < aptr[i + 1]; ++q) {
        int64_t at = fill[acol[q]]++;
        crow[at] = i;
        cval[at] = aval[q];
      }
  }
  // K = shift I + A P^{-1} A^T, lower triangle, as columns: kcp[j] ..
  // kcp[j+1] holds the rows i >= j (ascending) and values of column j.  Up to
  // kDenseAssembly rows K is summed in a dense m x m array (fast); above, as
  // one term a_ie w_e a_je per pair of constraints touching entry e, sorted
  // and summed per (column, row) key, so that a sparse K of any order needs
  // memory in proportion to those pairs only.
  constexpr int32_t kDenseAssembly = 8192;
  std::vector<int64_t> kcp(m + 1, 0);
  std::vector<int32_t> krow;
  std::vector<double> kval;
  if (m <= kDenseAssembly) {
    std::vector<double> K((size_t)m * m, 0.0);   // column-major, lower used
    for (int32_t i = 0; i < m; ++i) K[(size_t)i * m + i] = shift;
    for (int64_t e = 0; e < nE; ++e) {
      const double w = pinv[e];
      for (int64_t a = cptr[e]; a < cptr[e + 1]; ++a) {
        const int32_t i = crow[a];
        const double ai = cval[a] * w;
        for (int64_t bq = cptr[e]; bq <= a; ++bq) K[(size_t)crow[bq] * m + i] += ai * cval[bq];
      }
    }
    for (int32_t j = 0; j < m; ++j)
      for (int32_t i = j; i < m; ++i)
        if (K[(size_t)j * m + i] != 0.0) {
          krow.push_back(i);
          kval.push_back(K[(size_t)j * m + i]);
          kcp[j + 1]++;
        }
  } else {
    struct Term {
      int64_t key;   // j m + i
      double v;
    };
    std::vector<Term> terms;
    int64_t nt = m;
    for (int64_t e = 0; e < nE; ++e) nt += (cptr[e + 1] - cptr[e]) * (cptr[e + 1] - cptr[e] + 1) / 2;
    terms.reserve((size_t)nt);
    for (int32_t i = 0; i < m; ++i) terms.push_back({(int64_t)i * m + i, shift});
    for (int64_t e = 0; e < nE; ++e) {
      const double w = pinv[e];
      for (int64_t a = cptr[e]; a < cptr[e + 1]; ++a) {
        const int32_t i = crow[a];
        const double ai = cval[a] * w;
        for (int64_t bq = cptr[e]; bq <= a; ++bq) terms.push_back({(int64_t)crow[bq] * m + i, ai * cval[bq]});
      }
    }
    std::stable_sort(terms.begin(), terms.end(), [](const Term& x, const Term& y) { return x.key < y.key; });
    for (size_t t = 0; t < terms.size();) {
      size_t u = t;
      double v = 0.0;
      while (u < terms.size() && terms[u].key == terms[t].key) v += terms[u++].v;
      if (v != 0.0) {
        krow.push_back((int32_t)(terms[t].key % m));
        kval.push_back(v);
        kcp[terms[t].key / m + 1]++;
      }
      t = u;
    }
  }
  for (int32_t j = 0; j < m; ++j) kcp[j + 1] += kcp[j];
  const int64_t nnz = kcp[m];
  const double density = (double)nnz / (0.5 * (double)m * (m + 1));
  if (m <= 64 || (density > 0.2 && m <= 2048)) {
    f.dense = true;
    std::vector<double> K((size_t)m * m, 0.0);   // column-major, lower used
    for (int32_t j = 0; j < m; ++j)
      for (int64_t q = kcp[j]; q < kcp[j + 1]; ++q) K[(size_t)j * m + krow[q]] = kval[q];
    std::vector<double>& L = K;
    for (int32_t j = 0; j < m; ++j) {
      double d = L[(size_t)j * m + j];
      for (int32_t k = 0; k < j; ++k) d -= L[(size_t)k * m + j] * L[(size_t)k * m + j];
      if (!(d > 0.0)) return fail(err, CDCS_E_FACTOR, "Cholesky of the m x m matrix broke down (constraints linearly dependent on the pattern?)");
      const double ljj = std::sqrt(d);
      L[(size_t)j * m + j] = ljj;
      for (int32_t i = j + 1; i < m; ++i) {
        double s = L[(size_t)j * m + i];
        for (int32_t k = 0; k < j; ++k) s -= L[(size_t)k * m + i] * L[(size_t)k * m + j];
        L[(size_t)j * m + i] = s / ljj;
      }
      for (int32_t k = 0; k < j; ++k) L[(size_t)j * m + k] = 0.0;   // clear upper
    }
    f.Ld.swap(L);
    if (m <= kInvOrder) {
      // K^{-1} = L^{-T} L^{-1}: X = L^{-1} column by column (L x = e_c by
      // forward substitution), then X^T X
      std::vector<double> X((size_t)m * m, 0.0);
      for (int32_t c = 0; c < m; ++c) {
        double* x = &X[(size_t)c * m];
        x[c] = 1.0;
        for (int32_t j = c; j < m; ++j) {
          x[j] /= f.Ld[(size_t)j * m + j];
          for (int32_t i = j + 1; i < m; ++i) x[i] -= f.Ld[(size_t)j * m + i] * x[j];
        }
      }
      f.Kinv.assign((size_t)m * m, 0.0);
      for (int32_t c = 0; c < m; ++c)
        for (int32_t r = c; r < m; ++r) {
          double s = 0.0;
          for (int32_t k = r; k < m; ++k) s += X[(size_t)r * m + k] * X[(size_t)c * m + k];
          f.Kinv[(size_t)c * m + r] = s;
          f.Kinv[(size_t)r * m + c] = s;
        }
    }
    return 0;
  }
  // sparse: minimum-degree order, structure from the elimination game
  f.dense = false;
  std::vector<std::set<int32_t>> adj(m);
  for (int32_t j = 0; j < m; ++j)
    for (int64_t q = kcp[j]; q < kcp[j + 1]; ++q)
      if (krow[q] != j) {
        adj[krow[q]].insert(j);
        adj[j].insert(krow[q]);
      }
  std::vector<int32_t> order;
  std::vector<std::vector<int32_t>> higher;
  min_degree(m, adj, order, higher);
  std::vector<int32_t> pos(m);
  for (int32_t t = 0; t < m; ++t) pos[order[t]] = t;
  f.perm = order;                                   // Kp(i, j) = K(order[i], order[j])
  std::vector<std::vector<int32_t>> colrows(m);     // permuted rows > j of column j
  for (int32_t t = 0; t < m; ++t) {
    auto& cr = colrows[t];
    for (int32_t u : higher[order[t]]) cr.push_back(pos[u]);
    std::sort(cr.begin(), cr.end());
  }
  std::vector<std::vector<int32_t>> rowcols(m);     // columns k < r with L(r, k) != 0
  for (int32_t k = 0; k < m; ++k)
    for (int32_t r : colrows[k]) rowcols[r].push_back(k);
  std::vector<std::vector<double>> colvals(m);
  std::vector<double> work(m, 0.0);
  auto Kp = [&](int32_t i, int32_t j) {            // i >= j in permuted labels
    int32_t a = order[i], b = order[j];
    if (a < b) std::swap(a, b);
    const auto lo = krow.begin() + kcp[b], hi = krow.begin() + kcp[b + 1];
    const auto it = std::lower_bound(lo, hi, a);
    return (it != hi && *it == a) ? kval[it - krow.begin()] : 0.0;
  };
  f.diag.assign(m, 0.0);
  for (int32_t j = 0; j < m; ++j) {
    work[j] = Kp(j, j);
    for (int32_t r : colrows[j]) work[r] = Kp(r, j);
    for (int32_t k : rowcols[j]) {
      const auto& rows = colrows[k];
      const auto& vals = colvals[k];
      auto it = std::lower_bound(rows.begin(), rows.end(), j);
      size_t q = it - rows.begin();
      const double ljk = vals[q];
      work[j] -= ljk * ljk;
      for (size_t t = q + 1; t < rows.size(); ++t) work[rows[t]] -= vals[t] * ljk;
    }
    if (!(work[j] > 0.0)) return fail(err, CDCS_E_FACTOR, "sparse Cholesky of the m x m matrix broke down (constraints linearly dependent on the pattern?)");
    const double ljj = std::sqrt(work[j]);
    f.diag[j] = ljj;
    work[j] = 0.0;
    auto& cv = colvals[j];
    cv.resize(colrows[j].size());
    for (size_t t = 0; t < colrows[j].size(); ++t) {
      cv[t] = work[colrows[j][t]] / ljj;
      work[colrows[j][t]] = 0.0;
    }
  }
  // CSR of the strict lower factor (by row) and of L^T (by row = L by column)
  f.lptr.assign(m + 1, 0);
  for (int32_t k = 0; k < m; ++k)
    for (int32_t r : colrows[k]) f.lptr[r + 1]++;
  for (int32_t i = 0; i < m; ++i) f.lptr[i + 1] += f.lptr[i];
  f.lcol.resize(f.lptr[m]);
  f.lval.resize(f.lptr[m]);
  {
    std::vector<int32_t> fill(f.lptr.begin(), f.lptr.end() - 1);
    for (int32_t k = 0; k < m; ++k)
      for (size_t t = 0; t < colrows[k].size(); ++t) {
        int32_t r = colrows[k][t];
        f.lcol[fill[r]] = k;
        f.lval[fill[r]++] = colvals[k][t];
      }
  }
  f.uptr.assign(m + 1, 0);
  for (int32_t k = 0; k < m; ++k) f.uptr[k + 1] = f.uptr[k] + (int32_t)colrows[k].size();
  f.ucol.resize(f.uptr[m]);
  f.uval.resize(f.uptr[m]);
  for (int32_t k = 0; k < m; ++k)
    for (size_t t = 0; t < colrows[k].size(); ++t) {
      f.ucol[f.uptr[k] + t] = colrows[k][t];
      f.uval[f.uptr[k] + t] = colvals[k][t];
    }
  // level sets: forward (rows depend on smaller columns), backward (on larger)
  std::vector<int32_t> lev(m, 0);
  int32_t nlev = 0;
  for (int32_t i = 0; i < m; ++i) {
    int32_t l = 0;
    for (int32_t q = f.lptr[i]; q < f.lptr[i + 1]; ++q) l = std::max(l, lev[f.lcol[q]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  auto group = [&](std::vector<int32_t>& ptr, std::vector<int32_t>& rows, int32_t nl) {
    ptr.assign(nl + 1, 0);
    for (int32_t i = 0; i < m; ++i) ptr[lev[i] + 1]++;
    for (int32_t l = 0; l < nl; ++l) ptr[l + 1] += ptr[l];
    rows.resize(m);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int32_t i = 0; i < m; ++i) rows[fill[lev[i]]++] = i;
  };
  group(f.flev_ptr, f.flev_rows, nlev);
  // backward solve: row i of L^T depends on the larger rows it references
  std::fill(lev.begin(), lev.end(), 0);
  nlev = 0;
  for (int32_t i = m - 1; i >= 0; --i) {
    int32_t l = 0;
    for (int32_t q = f.uptr[i]; q < f.uptr[i + 1]; ++q) l = std::max(l, lev[f.ucol[q]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  group(f.blev_ptr, f.blev_rows, nlev);
  return 0;
}

int build_instance(const cdcs_problem& P, Instance& I, Error& err, int32_t method) {
  const int32_t n = P.n, m = P.m, p = P.p;
  if (n < 1 || m < 1 || p < 1) return fail(err, CDCS_E_ARG, "need n >= 1, m >= 1, p >= 1");
  if (!P.b || !P.clique_ptr || !P.clique_vtx) return fail(err, CDCS_E_ARG, "null b or clique arrays");
  if (P.c_nnz < 0 || P.a_nnz < 0) return fail(err, CDCS_E_ARG, "negative nnz");
  if (P.c_nnz > 0 && (!P.c_row || !P.c_col || !P.c_val)) return fail(err, CDCS_E_ARG, "null C arrays");
  if (P.a_nnz > 0 && (!P.a_con || !P.a_row || !P.a_col || !P.a_val))
    return fail(err, CDCS_E_ARG, "null A arrays");
  I.n = n;
  I.m = m;
  I.p = p;
  // ---- cliques (Section 2.1: vertices of C_k in natural order) ----
  if (P.clique_ptr[0] != 0) return fail(err, CDCS_E_CLIQUES, "clique_ptr[0] must be 0");
  std::vector<char> covered(n, 0);
  I.csize.resize(p);
  for (int32_t k = 0; k < p; ++k) {
    const int32_t a = P.clique_ptr[k], bnd = P.clique_ptr[k + 1];
    if (bnd <= a) return fail(err, CDCS_E_CLIQUES, "empty clique or decreasing clique_ptr");
    if (bnd - a > 1024) return fail(err, CDCS_E_CLIQUES, "clique larger than 1024 vertices");
    for (int32_t t = a; t < bnd; ++t) {
      const int32_t v = P.clique_vtx[t];
      if (v < 0 || v >= n) return fail(err, CDCS_E_CLIQUES, "clique vertex out of range");
      if (t > a && v <= P.clique_vtx[t - 1])
        return fail(err, CDCS_E_CLIQUES, "clique vertices must be strictly increasing");
      covered[v] = 1;
    }
    I.csize[k] = bnd - a;
  }
  for (int32_t v = 0; v < n; ++v)
    if (!covered[v]) return fail(err, CDCS_E_CLIQUES, "vertex " + std::to_string(v) + " is in no clique");
  if (P.clique_parent) {
    // induced-subtree property: cliques containing a vertex form a subtree
    std::vector<int32_t> cnt(n, 0), edg(n, 0), mark(n, -1);
    for (int32_t k = 0; k < p; ++k) {
      const int32_t par = P.clique_parent[k];
      if (par < -1 || par >= p || par == k) return fail(err, CDCS_E_CLIQUES, "bad clique parent");
      for (int32_t t = P.clique_ptr[k]; t < P.clique_ptr[k + 1]; ++t) cnt[P.clique_vtx[t]]++;
      if (par >= 0) {
        for (int32_t t = P.clique_ptr[par]; t < P.clique_ptr[par + 1]; ++t) mark[P.clique_vtx[t]] = k;
        for (int32_t t = P.clique_ptr[k]; t < P.clique_ptr[k + 1]; ++t)
          if (mark[P.clique_vtx[t]] == k) edg[P.clique_vtx[t]]++;
      }
    }
    for (int32_t v = 0; v < n; ++v)
      if (edg[v] != cnt[v] - 1)
        return fail(err, CDCS_E_CLIQUES, "clique tree violates the running-intersection property");
  }
  // ---- E' = union of C_k x C_k, lower entries, sorted by (col, row) ----
  int64_t total_slots = 0;
  I.slot_off.resize(p + 1);
  I.slot_off[0] = 0;
  for (int32_t k = 0; k < p; ++k) {
    total_slots += (int64_t)I.csize[k] * (I.csize[k] + 1) / 2;
    I.slot_off[k + 1] = total_slots;
  }
  if (total_slots >= (int64_t)INT32_MAX) return fail(err, CDCS_E_ARG, "too many clique entries");
  I.ns = total_slots;
  std::vector<int64_t> keys(total_slots);
  {
    int64_t at = 0;
    for (int32_t k = 0; k < p; ++k) {
      const int32_t* v = P.clique_vtx + P.clique_ptr[k];
      const int32_t K = I.csize[k];
      for (int32_t bb = 0; bb < K; ++bb)
        for (int32_t a = bb; a < K; ++a) keys[at++] = (int64_t)v[bb] * n + v[a];
    }
  }
  std::vector<int64_t> ukeys(keys);
  std::sort(ukeys.begin(), ukeys.end());
  ukeys.erase(std::unique(ukeys.begin(), ukeys.end()), ukeys.end());
  I.nE = (int64_t)ukeys.size();
  I.erow.resize(I.nE);
  I.ecol.resize(I.nE);
  for (int64_t e = 0; e < I.nE; ++e) {
    I.ecol[e] = (int32_t)(ukeys[e] / n);
    I.erow[e] = (int32_t)(ukeys[e] % n);
  }
  auto find = [&](int64_t key) -> int64_t {
    auto it = std::lower_bound(ukeys.begin(), ukeys.end(), key);
    if (it == ukeys.end() || *it != key) return -1;
    return it - ukeys.begin();
  };
  // ---- H: slot -> entry (Section 3.1, H_k = E_k (x) E_k restricted to svec) ----
  I.slot2ent.resize(total_slots);
  I.D.assign(I.nE, 0);
  for (int64_t s = 0; s < total_slots; ++s) {
    const int64_t e = find(keys[s]);
    I.slot2ent[s] = (int32_t)e;
    I.D[e]++;
  }
  // ---- c = svec(C), A = [svec(A_i)]^T ----
  I.c.assign(I.nE, 0.0);
  for (int64_t t = 0; t < P.c_nnz; ++t) {
    const int32_t r = P.c_row[t], q = P.c_col[t];
    const double v = P.c_val[t];
    if (r < 0 || r >= n || q < 0 || q > r) return fail(err, CDCS_E_ARG, "C entry not in the lower triangle");
    if (!finite(v)) return fail(err, CDCS_E_NONFINITE, "non-finite value in C");
    const int64_t e = find((int64_t)q * n + r);
    if (e < 0) return fail(err, CDCS_E_PATTERN, "C entry outside the chordal pattern");
    I.c[e] += (r == q) ? v : kSqrt2 * v;
  }
  struct Trip { int32_t i; int32_t e; double v; };
  std::vector<Trip> trips;
  trips.reserve(P.a_nnz);
  for (int64_t t = 0; t < P.a_nnz; ++t) {
    const int32_t i = P.a_con[t], r = P.a_row[t], q = P.a_col[t];
    const double v = P.a_val[t];
    if (i < 0 || i >= m) return fail(err, CDCS_E_ARG, "constraint index out of range");
    if (r < 0 || r >= n || q < 0 || q > r) return fail(err, CDCS_E_ARG, "A entry not in the lower triangle");
    if (!finite(v)) return fail(err, CDCS_E_NONFINITE, "non-finite value in A");
    const int64_t e = find((int64_t)q * n + r);
    if (e < 0) return fail(err, CDCS_E_PATTERN, "A entry outside the chordal pattern");
    trips.push_back({i, (int32_t)e, (r == q) ? v : kSqrt2 * v});
  }
  std::sort(trips.begin(), trips.end(), [](const Trip& x, const Trip& y) {
    return x.i != y.i ? x.i < y.i : x.e < y.e;
  });
  I.aptr.assign(m + 1, 0);
  for (size_t t = 0; t < trips.size();) {
    size_t u = t;
    double v = 0.0;
    while (u < trips.size() && trips[u].i == trips[t].i && trips[u].e == trips[t].e) v += trips[u++].v;
    I.acol.push_back(trips[t].e);
    I.aval.push_back(v);
    I.aptr[trips[t].i + 1]++;
    t = u;
  }
  for (int32_t i = 0; i < m; ++i) I.aptr[i + 1] += I.aptr[i];
  if ((int64_t)I.acol.size() >= (int64_t)INT32_MAX) return fail(err, CDCS_E_ARG, "A too large");
  I.b.assign(P.b, P.b + m);
  for (double v : I.b)
    if (!finite(v)) return fail(err, CDCS_E_NONFINITE, "non-finite value in b");
  if (method != 0) {
    // primal-only / dual-only ADMM: step 1 of both reduces to the m x m
    // matrix A D^{-1} A^T (no Sherman-Morrison data)
    std::vector<double> dinv(I.nE);
    for (int64_t e = 0; e < I.nE; ++e) dinv[e] = 1.0 / (double)I.D[e];
    int rc = factor_K(m, I.aptr, I.acol, I.aval, dinv, I.fac, err, 0.0);
    if (rc) return rc;
    I.zt_x.assign(I.nE, 0.0);
    I.atzy.assign(I.nE, 0.0);
    I.zt_y.assign(m, 0.0);
    double nb = 0.0, nc = 0.0;
    for (int64_t e = 0; e < I.nE; ++e) nc += I.c[e] * I.c[e];
    for (int32_t i = 0; i < m; ++i) nb += I.b[i] * I.b[i];
    I.den = 1.0;
    I.ctzx = I.btzy = 0.0;
    I.nb = std::sqrt(nb);
    I.nc = std::sqrt(nc);
    return 0;
  }
  // ---- factor of the inner matrix (eqs. ThirdBlkElm, FactorizationMatrix) ----
  std::vector<double> pinv(I.nE);
  for (int64_t e = 0; e < I.nE; ++e) pinv[e] = 1.0 / (1.0 + 0.5 * I.D[e]);
  int rc = factor_K(m, I.aptr, I.acol, I.aval, pinv, I.fac, err, 1.0);
  if (rc) return rc;
  // ---- Sherman-Morrison data (eq. MatrixInverseResult) ----
  // zeta = (c, 0, -b, 0); M^{-1} zeta through the same eliminations:
  //   w = K^{-1}(A P^{-1} c + b), zt_x = P^{-1}(c - A^T w), zt_y = -w,
  //   s/v parts = +-H zt_x / 2 (never stored).
  std::vector<double> g(m, 0.0);
  for (int32_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int32_t q = I.aptr[i]; q < I.aptr[i + 1]; ++q) s += I.aval[q] * pinv[I.acol[q]] * I.c[I.acol[q]];
    g[i] = s + I.b[i];
  }
  I.fac.solve(g);
  std::vector<double> atw(I.nE, 0.0);
  for (int32_t i = 0; i < m; ++i)
    for (int32_t q = I.aptr[i]; q < I.aptr[i + 1]; ++q) atw[I.acol[q]] += I.aval[q] * g[i];
  I.zt_x.resize(I.nE);
  I.atzy.resize(I.nE);
  I.zt_y.resize(m);
  double ctzx = 0.0, btzy = 0.0, nb = 0.0, nc = 0.0;
  for (int64_t e = 0; e < I.nE; ++e) {
    I.zt_x[e] = pinv[e] * (I.c[e] - atw[e]);
    I.atzy[e] = -atw[e];
    ctzx += I.c[e] * I.zt_x[e];
    nc += I.c[e] * I.c[e];
  }
  for (int32_t i = 0; i < m; ++i) {
    I.zt_y[i] = -g[i];
    btzy += I.b[i] * I.zt_y[i];
    nb += I.b[i] * I.b[i];
  }
  I.ctzx = ctzx;
  I.btzy = btzy;
  I.den = 1.0 + ctzx - btzy;
  I.nb = std::sqrt(nb);
  I.nc = std::sqrt(nc);
  return 0;
}

}  // namespace cdcs
