// Host-side plan of a (batched) HSDE-ADMM solve: everything cached before the
// iterations start (Sections 4.2-4.3: the factor of the inner matrix and the
// Sherman-Morrison data), laid out as concatenated device arrays.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cdcs.h"

namespace cdcs {

struct Error {
  int code;
  std::string msg;
};

// Cholesky factor of K = I + A P^{-1} A^T for one instance (m x m).
constexpr int32_t kInvOrder = 512;

struct Factor {
  int32_t m = 0;
  bool dense = true;
  // dense: column-major lower m x m; for m <= kInvOrder also K^{-1} (m x m,
  // both triangles), so that the device solve is one matrix-vector product
  std::vector<double> Ld;
  std::vector<double> Kinv;
  // sparse: Kp = K[perm][:, perm] = L L^T
  std::vector<int32_t> perm;
  std::vector<double> diag;                       // L_ii
  std::vector<int32_t> lptr, lcol;                // strict lower, CSR by row
  std::vector<double> lval;
  std::vector<int32_t> uptr, ucol;                // strict upper of L^T, CSR by row (= L by column)
  std::vector<double> uval;
  std::vector<int32_t> flev_ptr, flev_rows;       // forward level sets
  std::vector<int32_t> blev_ptr, blev_rows;       // backward level sets
  void solve(std::vector<double>& g) const;       // in place K^{-1} g (host)
};

struct Instance {
  int32_t n = 0, m = 0, p = 0;
  int64_t nE = 0, ns = 0;
  // E' lower entries, canonical (col, row) order
  std::vector<int32_t> erow, ecol;
  std::vector<double> c;                          // svec(C)
  std::vector<double> b;
  // A as CSR over local entries
  std::vector<int32_t> aptr, acol;
  std::vector<double> aval;
  // slots: clique k occupies [slot_off[k], slot_off[k+1])
  std::vector<int64_t> slot_off;
  std::vector<int32_t> csize;
  std::vector<int32_t> slot2ent;                  // local entry of each slot
  std::vector<int32_t> D;                         // number of cliques covering each entry
  Factor fac;
  // Sherman-Morrison cache (eq. MatrixInverseResult)
  std::vector<double> zt_x, zt_y, atzy;           // M^{-1} zeta (x, y parts), A^T zt_y
  double den = 1.0, ctzx = 0.0, btzy = 0.0, nb = 0.0, nc = 0.0;
};

// Build one instance (validation, E', H, A, factor, Sherman-Morrison data).
// method 0 = the self-dual embedding (factor of I + A P^{-1} A^T); 1, 2 =
// the primal-only / dual-only ADMM (factor of A D^{-1} A^T, no
// Sherman-Morrison data).  Returns 0 or a negative CDCS_E_* code with err
// filled.
int build_instance(const cdcs_problem& P, Instance& out, Error& err, int32_t method = 0);

// Dense Cholesky / sparse factor helpers (exposed for tests of the host code)
// K = shift I + A diag(pinv) A^T (shift 1: the self-dual method; 0: the
// primal-only / dual-only methods)
int factor_K(int32_t m, const std::vector<int32_t>& aptr, const std::vector<int32_t>& acol,
             const std::vector<double>& aval, const std::vector<double>& pinv, Factor& f, Error& err,
             double shift = 1.0);

}  // namespace cdcs
