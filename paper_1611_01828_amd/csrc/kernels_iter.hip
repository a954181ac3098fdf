// Per-iteration streaming kernels of step 1 (the affine projection, Sections
// 4.2-4.3) and the fused vector updates / residual reductions.
//
// With h = r = w = 0 (they stay exactly zero, step (Step3)) and
// omega = u + v~ = (x, s + z, y, v, tau + kappa), step 1 in the eliminated
// form reads (eq. MatrixInverse: t = omega_12 - omega_3 zeta, zeta = (c,0,-b,0);
// eq. SecBlkEliResult/ThirdBlkElm eliminated onto the first block; eq.
// FactorizationMatrix inverted by the matrix inversion lemma with P = I + D/2
// and K = I + A P^{-1} A^T):
//
//   r0  = x - omega_3 c + H^T(s + z + v)/2                     k_r0
//   g'  = A P^{-1} r0 - y - omega_3 b                          k_spmv_a
//   w'  = K^{-1} g'                                            k_trsv
//   p_x = P^{-1}(r0 - A^T w'),  p_y = -w'                      k_spmv_at
//   gamma = (c^T p_x + b^T w') / (1 + zeta^T M^{-1} zeta)      k_scalar1 (eq. MatrixInverseResult)
//   x+ = p_x - gamma zt_x,  y+ = -w' - gamma zt_y              k_update_e / k_update_r
//   u_tau = omega_3 + c^T x+ - b^T y+                          (eq. FirstBlockElimination)
//   tau+ = max(0, u_tau - kappa), kappa+ = tau+ - (u_tau - kappa)   (Step2/Step3)
//
// The clique blocks (u_s - z, v+ and the PSD projection) are handled by the
// cone kernels.  Residual norms reuse these intermediates: A x+ = w' + y +
// omega_3 b + gamma (b + zt_y), A^T y+ = -A^T w' - gamma A^T zt_y and
// H^T v+ = H^T(s+z+v)/2 - D x+ / 2.
//
// Relaxed steps 2-3 (alpha != 1, O'Donoghue et al. 2016): x+, y+, v+ and the
// tau argument are u + alpha (u_hat - u), so each product of the new iterate
// is the same blend of the product of u_hat above and that of the previous
// iterate; A x, A^T y and H^T v of the previous iterate are summed in k_spmv_a,
// k_spmv_at and k_r0, which read those index lists anyway (RELAX templates).
#include "device.h"

namespace cdcs {

template <bool RELAX>
__global__ __launch_bounds__(kThreads) void k_r0(DevPlan d) {
  const int4 bd = d.eblk[blockIdx.x];
  const int inst = bd.x;
  if (d.st[inst * kNst + ST_FROZEN]) return;
  const double om3 = d.sc[inst * kNsc + SC_TAU] + d.sc[inst * kNsc + SC_KAPPA];
  for (int e = bd.y + threadIdx.x; e < bd.z; e += kThreads) {
    // the entry's slots in batches of 4 with clamped indices, so that a
    // batch's loads are in flight together; terms added in slot order
    double acc = 0.0, accv = 0.0;
    const int k0 = d.ent_sptr[e], k1 = d.ent_sptr[e + 1];
    for (int kb = k0; kb < k1; kb += 4) {
      int sl[4];
      double sv[4], zv[4], vv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) sl[u] = d.ent_slots[min(kb + u, k1 - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sv[u] = d.s[sl[u]];
        zv[u] = d.z[sl[u]];
        vv[u] = d.v[sl[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (kb + u < k1) {
          acc += sv[u] + zv[u] + vv[u];
          if (RELAX) accv += vv[u];
        }
    }
    if (RELAX) d.hvo[e] = accv;
    const double hs = 0.5 * acc;
    const double r0 = d.x[e] - om3 * d.c[e] + hs;
    d.hsum[e] = hs;
    d.q[e] = d.pinv[e] * r0;
  }
}

// one wavefront per constraint row: workgroup (b, y) takes rows
// 4 y .. 4 y + 3 of row block b
template <bool RELAX>
__global__ __launch_bounds__(kThreads) void k_spmv_a(DevPlan d) {
  const int4 bd = d.rblk[blockIdx.x];
  const int inst = bd.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r = bd.y + blockIdx.y * (kThreads / 64) + wid;
  if (r >= bd.z || d.st[inst * kNst + ST_FROZEN]) return;
  const double om3 = d.sc[inst * kNsc + SC_TAU] + d.sc[inst * kNsc + SC_KAPPA];
  {
    // batches of kBatch nonzeros per lane with clamped indices, so that all
    // loads of a batch are in flight together (a bounds test per load would
    // serialise them); each lane still sums its nonzeros q, q + 64, ... in order
    constexpr int kBatch = 8;
    double acc = 0.0, accx = 0.0;
    const int q0 = d.a_ptr[r], q1 = d.a_ptr[r + 1];
    for (int qb = q0; qb < q1; qb += 64 * kBatch) {
      int col[kBatch];
      double av[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int qc = min(qb + 64 * u + lane, q1 - 1);
        col[u] = d.a_col[qc];
        av[u] = d.a_val[qc];
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const double m = (qb + 64 * u + lane < q1) ? av[u] : 0.0;
        acc += m * d.q[col[u]];
        if (RELAX) accx += m * d.x[col[u]];   // x is still the previous iterate here
      }
    }
    acc = wave_sum(acc);
    if (RELAX) accx = wave_sum(accx);
    if (lane == 0) {
      d.g[r] = acc - d.y[r] - om3 * d.b[r];
      if (RELAX) d.axo[r] = accx;
    }
  }
}

// K w' = g' for one instance per workgroup: K = L L^T (dense column-major L)
// or Kp = L L^T in a minimum-degree order with level-scheduled rows.
constexpr int kTrsvThreads = 256;
constexpr int kTrsvLds = 8192;
constexpr int kTrsvDense = 2048;   // largest m of the dense form
static_assert(3 * kTrsvDense <= kTrsvLds, "the dense sweeps keep three vectors in LDS");

// One column-oriented sweep of a dense triangular solve held in LDS:
// for j in order, x_j = rhs_j / dg_j and rhs_i -= M(i, j) x_j for the rows
// i after j (forward: M = L, rows below; backward: M = L^T stored as its own
// column-major matrix, rows above, so that both sweeps read columns).  Thread
// t owns rows t + 256 r (r < R); the next PD columns it needs are kept in
// registers, loaded PD columns ahead, so one barrier per column remains.
template <int R, int PD, bool FWD>
__device__ __forceinline__ void trsv_sweep(const double* M, int m, double* rhs, double* out, const double* dg) {
  const int tid = threadIdx.x;
  double ring[PD][R];
  auto col_of = [&](int k) { return FWD ? min(k, m - 1) : max(m - 1 - k, 0); };
#pragma unroll
  for (int p = 0; p < PD; ++p)
#pragma unroll
    for (int r = 0; r < R; ++r) ring[p][r] = M[(size_t)col_of(p) * m + min(tid + kTrsvThreads * r, m - 1)];
  for (int k0 = 0; k0 < m; k0 += PD) {
#pragma unroll
    for (int p = 0; p < PD; ++p) {
      const int k = k0 + p;
      if (k < m) {
        const int j = FWD ? k : m - 1 - k;
        const double xj = rhs[j] / dg[j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = tid + kTrsvThreads * r;
          if (i < m && (FWD ? i > j : i < j)) rhs[i] -= ring[p][r] * xj;
        }
        if (tid == 0) out[j] = xj;
        const int jn = col_of(k + PD);
#pragma unroll
        for (int r = 0; r < R; ++r) ring[p][r] = M[(size_t)jn * m + min(tid + kTrsvThreads * r, m - 1)];
      }
      __syncthreads();
    }
  }
}

template <int R, int PD>
__global__ __launch_bounds__(kTrsvThreads) void k_trsv(DevPlan d) {
  __shared__ double zl[kTrsvLds];
  __shared__ double red[kTrsvThreads / 64 + 1];
  const int inst = blockIdx.x;
  if (d.st[inst * kNst + ST_FROZEN]) return;
  const int r0 = d.row_off[inst];
  const int m = d.row_off[inst + 1] - r0;
  const int tid = threadIdx.x;
  if (d.f_mode[inst] == 2) {
    // w' = K^{-1} g' with K^{-1} cached at setup: a product with no chain of
    // dependent column steps; K^{-1} read column by column (coalesced), g'
    // broadcast from LDS, loads 32 columns at a time (clamped, then masked)
    const double* Ki = d.f_Kinv + d.f_dense_off[inst];
    for (int i = tid; i < m; i += kTrsvThreads) zl[i] = d.g[r0 + i];
    __syncthreads();
    double bw = 0.0;
    for (int i = tid; i < m; i += kTrsvThreads) {
      double acc = 0.0;
      for (int j0 = 0; j0 < m; j0 += 32) {
        double kv[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) kv[u] = Ki[(size_t)min(j0 + u, m - 1) * m + i];
#pragma unroll
        for (int u = 0; u < 32; ++u) acc += (j0 + u < m) ? kv[u] * zl[min(j0 + u, m - 1)] : 0.0;
      }
      d.w[r0 + i] = acc;
      bw += d.b[r0 + i] * acc;
    }
    bw = block_sum<kTrsvThreads>(bw, red);
    if (tid == 0) d.sc[inst * kNsc + SC_BW] = bw;
    return;
  }
  if (d.f_mode[inst] == 0) {
    // zl: right-hand side (then the result); zf: forward result; dg: diagonal
    const double* L = d.f_Ld + d.f_dense_off[inst];
    const double* Lt = d.f_Ldt + d.f_dense_off[inst];
    double* zf = zl + kTrsvDense;
    double* dg = zl + 2 * kTrsvDense;
    for (int i = tid; i < m; i += kTrsvThreads) {
      zl[i] = d.g[r0 + i];
      dg[i] = L[(size_t)i * m + i];
    }
    __syncthreads();
    if (m > 0) {
      trsv_sweep<R, PD, true>(L, m, zl, zf, dg);     // L z = g
      trsv_sweep<R, PD, false>(Lt, m, zf, zl, dg);   // L^T w = z
    }
    double bw = 0.0;
    for (int i = tid; i < m; i += kTrsvThreads) {
      d.w[r0 + i] = zl[i];
      bw += d.b[r0 + i] * zl[i];
    }
    bw = block_sum<kTrsvThreads>(bw, red);
    if (tid == 0) d.sc[inst * kNsc + SC_BW] = bw;
    return;
  }
  // sparse, permuted: z = g[perm], in LDS up to kTrsvLds rows, above in
  // the instance's slice of the global vector trsv_z (the barriers between
  // levels order its writes and reads within the workgroup)
  double* z = (m <= kTrsvLds) ? zl : d.trsv_z + r0;
  const int32_t* perm = d.f_perm + r0;
  const double* dg = d.f_diag + r0;
  const int32_t* lptr = d.f_lptr + r0 + inst;
  const int32_t* uptr = d.f_uptr + r0 + inst;
  for (int i = tid; i < m; i += kTrsvThreads) z[i] = d.g[r0 + perm[i]];
  __syncthreads();
  {
    const int l0 = d.f_flev_off[inst], l1 = d.f_flev_off[inst + 1];
    for (int l = l0; l < l1; ++l) {
      const int a = d.f_flev_ptr[l], bnd = d.f_flev_ptr[l + 1];
      for (int t = a + tid; t < bnd; t += kTrsvThreads) {
        const int i = d.f_flev_rows[t];
        double sacc = z[i];
        for (int q = lptr[i]; q < lptr[i + 1]; ++q) sacc -= d.f_lval[q] * z[d.f_lcol[q]];
        z[i] = sacc / dg[i];
      }
      __syncthreads();
    }
  }
  {
    const int l0 = d.f_blev_off[inst], l1 = d.f_blev_off[inst + 1];
    for (int l = l0; l < l1; ++l) {
      const int a = d.f_blev_ptr[l], bnd = d.f_blev_ptr[l + 1];
      for (int t = a + tid; t < bnd; t += kTrsvThreads) {
        const int i = d.f_blev_rows[t];
        double sacc = z[i];
        for (int q = uptr[i]; q < uptr[i + 1]; ++q) sacc -= d.f_uval[q] * z[d.f_ucol[q]];
        z[i] = sacc / dg[i];
      }
      __syncthreads();
    }
  }
  double bw = 0.0;
  for (int i = tid; i < m; i += kTrsvThreads) {
    const int r = r0 + perm[i];
    d.w[r] = z[i];
    bw += d.b[r] * z[i];
  }
  bw = block_sum<kTrsvThreads>(bw, red);
  if (tid == 0) d.sc[inst * kNsc + SC_BW] = bw;
}

// A^T w' from the sliced-ELL copy of A^T: each wave takes chunks of 64
// entries of the block and steps through their nonzeros together (each
// entry's nonzeros in ascending row order, as in the CSR form).  The chunks
// hold the block's entries in sorted order, so the per-entry operands and
// results go through LDS: read and written in entry order (coalesced),
// addressed in chunk order.
template <bool RELAX>
__global__ __launch_bounds__(kThreads) void k_spmv_at(DevPlan d) {
  static_assert(kEntChunk <= 1024, "an entry block fits the LDS staging");
  __shared__ double red[kThreads / 64 + 1];
  __shared__ double s0[1024], s1[1024];   // q then p_x; P^{-1} then A^T w'
  __shared__ double s2[RELAX ? 1024 : 1];  // A^T y of the previous iterate
  const int4 bd = d.eblk[blockIdx.x];
  const int inst = bd.x;
  if (d.st[inst * kNst + ST_FROZEN]) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int n = bd.z - bd.y;
  const int nch = (n + 63) >> 6;
  const int c0 = d.at_choff[blockIdx.x];
  for (int l = threadIdx.x; l < n; l += kThreads) {
    s0[l] = d.q[bd.y + l];
    s1[l] = d.pinv[bd.y + l];
  }
  __syncthreads();
  for (int c = wid; c < nch; c += kThreads / 64) {
    const int ch = c0 + c;
    const int e = d.at_sent[(size_t)ch * 64 + lane];
    const int len = d.at_chlen[ch];
    const int32_t* srow = d.at_srow + d.at_chptr[ch] + lane;
    const double* sval = d.at_sval + d.at_chptr[ch] + lane;
    double acc = 0.0, accy = 0.0;
#pragma unroll 4
    for (int k = 0; k < len; ++k) {
      const int row = srow[(size_t)k * 64];
      const double av = sval[(size_t)k * 64];
      acc += av * d.w[row];
      if (RELAX) accy += av * d.y[row];   // y is still the previous iterate here
    }
    if (e < 0) continue;
    const int l = e - bd.y;
    if (RELAX) s2[l] = accy;
    s0[l] = s0[l] - s1[l] * acc;   // p_x
    s1[l] = acc;
  }
  __syncthreads();
  double cpx = 0.0;
  for (int l = threadIdx.x; l < n; l += kThreads) {
    const int e = bd.y + l;
    const double px = s0[l];
    d.px[e] = px;
    d.atw[e] = s1[l];
    if (RELAX) d.atyo[e] = s2[l];
    cpx += d.c[e] * px;
  }
  cpx = block_sum<kThreads>(cpx, red);
  if (threadIdx.x == 0) d.part_e[blockIdx.x * 4 + 0] = cpx;
}

// gamma of eq. (MatrixInverseResult), u_tau of eq. (FirstBlockElimination),
// and the R_+ parts of steps 2-3.
__global__ __launch_bounds__(64) void k_scalar1(DevPlan d) {
  const int inst = blockIdx.x;
  if (d.st[inst * kNst + ST_FROZEN]) return;
  double acc = 0.0;
  for (int b = d.eblk_off[inst] + threadIdx.x; b < d.eblk_off[inst + 1]; b += 64) acc += d.part_e[b * 4 + 0];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) {
    double* sc = d.sc + inst * kNsc;
    const double tau = sc[SC_TAU], kap = sc[SC_KAPPA];
    const double om3 = tau + kap;
    const double bw = sc[SC_BW];
    const double gam = (acc + bw) / sc[SC_DEN];
    const double cx = acc - gam * sc[SC_CTZX];       // c^T x+
    const double by = -bw - gam * sc[SC_BTZY];       // b^T y+
    const double ut = om3 + cx - by;
    const double ub = d.relax ? tau + d.alpha * (ut - tau) : ut;   // relaxed tau argument
    const double tn = fmax(0.0, ub - kap);
    sc[SC_CPX] = acc;
    sc[SC_GAMMA] = gam;
    sc[SC_OMEGA3] = om3;
    sc[SC_UTAU] = ut;
    sc[SC_TAU] = tn;
    sc[SC_KAPPA] = kap - ub + tn;
  }
}

template <bool RELAX>
__global__ __launch_bounds__(kThreads) void k_update_e(DevPlan d) {
  __shared__ double red[kThreads / 64 + 1];
  const int4 bd = d.eblk[blockIdx.x];
  const int inst = bd.x;
  if (d.st[inst * kNst + ST_FROZEN]) return;
  const double* sc = d.sc + inst * kNsc;
  const double gam = sc[SC_GAMMA], tau = sc[SC_TAU];
  const double al = d.alpha;
  double d2 = 0.0, p2 = 0.0, cx = 0.0;
  for (int e = bd.y + threadIdx.x; e < bd.z; e += kThreads) {
    const double xh = d.px[e] - gam * d.zt_x[e];   // u_hat_x
    double xn, lin;
    if (!RELAX) {
      xn = xh;
      // A^T y+ + H^T v+  (dual-feasibility row of eq. DualFeasible)
      lin = -d.atw[e] - gam * d.atzy[e] + d.hsum[e] - d.halfD[e] * xn;
    } else {
      const double xo = d.x[e], ao = d.atyo[e], ho = d.hvo[e];
      xn = xo + al * (xh - xo);
      const double aty = ao + al * ((-d.atw[e] - gam * d.atzy[e]) - ao);
      const double hv = ho + al * ((d.hsum[e] - d.halfD[e] * xh) - ho);
      lin = aty + hv;
      d.xh[e] = xh;
    }
    const double ce = d.c[e];
    const double dr = lin - tau * ce;
    d.x[e] = xn;
    d2 += dr * dr;
    p2 += lin * lin;
    cx += ce * xn;
  }
  d2 = block_sum<kThreads>(d2, red);
  p2 = block_sum<kThreads>(p2, red);
  cx = block_sum<kThreads>(cx, red);
  if (threadIdx.x == 0) {
    double* pe = d.part_e + blockIdx.x * 4;
    pe[1] = d2;
    pe[2] = p2;
    pe[3] = cx;
  }
}

template <bool RELAX>
__global__ __launch_bounds__(kThreads) void k_update_r(DevPlan d) {
  __shared__ double red[kThreads / 64 + 1];
  const int4 bd = d.rblk[blockIdx.x];
  const int inst = bd.x;
  if (d.st[inst * kNst + ST_FROZEN]) return;
  const double* sc = d.sc + inst * kNsc;
  const double gam = sc[SC_GAMMA], tau = sc[SC_TAU], om3 = sc[SC_OMEGA3];
  const double al = d.alpha;
  double p2 = 0.0, a2 = 0.0, by = 0.0;
  for (int r = bd.y + threadIdx.x; r < bd.z; r += kThreads) {
    const double br = d.b[r], ztr = d.zt_y[r], wr = d.w[r], yo = d.y[r];
    // A u_hat_x = A p_x - gamma A zt_x = (w' + y + omega_3 b) + gamma (b + zt_y)
    double ax = wr + yo + om3 * br + gam * (br + ztr);
    double yn = -wr - gam * ztr;                     // u_hat_y
    if (RELAX) {
      const double ao = d.axo[r];
      ax = ao + al * (ax - ao);
      yn = yo + al * (yn - yo);
    }
    d.y[r] = yn;
    const double pr = ax - tau * br;
    p2 += pr * pr;
    a2 += ax * ax;
    by += br * yn;
  }
  p2 = block_sum<kThreads>(p2, red);
  a2 = block_sum<kThreads>(a2, red);
  by = block_sum<kThreads>(by, red);
  if (threadIdx.x == 0) {
    double* pr = d.part_r + blockIdx.x * 4;
    pr[0] = p2;
    pr[1] = a2;
    pr[2] = by;
  }
}

// Residuals, termination and infeasibility tests (O'Donoghue et al. 2016
// normalisation of the KKT rows of eqs. PrimalFeasible, DualFeasible,
// ZeroGap); stop = 1 freezes an instance once it has an outcome.
__global__ __launch_bounds__(64) void k_scalar2(DevPlan d, double eps_tol, int32_t max_iter, int32_t stop) {
  const int inst = blockIdx.x;
  int32_t* st = d.st + inst * kNst;
  if (st[ST_FROZEN]) return;
  const int lane = threadIdx.x;
  double e1 = 0, e2 = 0, e3 = 0, r0 = 0, r1 = 0, r2 = 0, c0 = 0, c1 = 0;
  for (int b = d.eblk_off[inst] + lane; b < d.eblk_off[inst + 1]; b += 64) {
    e1 += d.part_e[b * 4 + 1];
    e2 += d.part_e[b * 4 + 2];
    e3 += d.part_e[b * 4 + 3];
  }
  for (int b = d.rblk_off[inst] + lane; b < d.rblk_off[inst + 1]; b += 64) {
    r0 += d.part_r[b * 4 + 0];
    r1 += d.part_r[b * 4 + 1];
    r2 += d.part_r[b * 4 + 2];
  }
  for (int k = d.clq_off[inst] + lane; k < d.clq_off[inst + 1]; k += 64) {
    c0 += d.part_c[k * 2 + 0];
    c1 += d.part_c[k * 2 + 1];
  }
  e1 = wave_sum(e1);
  e2 = wave_sum(e2);
  e3 = wave_sum(e3);
  r0 = wave_sum(r0);
  r1 = wave_sum(r1);
  r2 = wave_sum(r2);
  c0 = wave_sum(c0);
  c1 = wave_sum(c1);
  if (lane != 0) return;
  double* sc = d.sc + inst * kNsc;
  const double tau = sc[SC_TAU];
  const double cx = e3, by = r2;
  const double pri2 = r0 + c0, dua2 = e1 + c1, pinf2 = e2 + c1, dinf2 = r1 + c0;
  double ep = INFINITY, ed = INFINITY, eg = INFINITY;
  if (tau > 0.0) {
    ep = sqrt(pri2) / (tau * (1.0 + sc[SC_NB]));
    ed = sqrt(dua2) / (tau * (1.0 + sc[SC_NC]));
  }
  const double gden = tau + fabs(cx) + fabs(by);
  if (gden > 0.0) eg = fabs(cx - by) / gden;
  int status = 0;
  if (tau > 0.0 && ep <= eps_tol && ed <= eps_tol && eg <= eps_tol) status = 1;
  else if (by > 0.0 && sqrt(pinf2) <= eps_tol * by) status = 2;
  else if (cx < 0.0 && sqrt(dinf2) <= eps_tol * (-cx)) status = 3;
  sc[SC_EPS_P] = ep;
  sc[SC_EPS_D] = ed;
  sc[SC_EPS_G] = eg;
  sc[SC_CX] = cx;
  sc[SC_BY] = by;
  sc[SC_PRI2] = pri2;
  sc[SC_DUA2] = dua2;
  sc[SC_PINF2] = pinf2;
  sc[SC_DINF2] = dinf2;
  const int it = st[ST_ITER] + 1;
  st[ST_ITER] = it;
  st[ST_WARM] = 1;
  if (stop && status == 0 && it >= max_iter) status = 4;
  st[ST_STATUS] = status;
  if (stop && status != 0) st[ST_FROZEN] = 1;
}

void launch_r0(const DevPlan& d, hipStream_t st) {
  if (d.relax) hipLaunchKernelGGL(k_r0<true>, dim3(d.n_eblk), dim3(kThreads), 0, st, d);
  else hipLaunchKernelGGL(k_r0<false>, dim3(d.n_eblk), dim3(kThreads), 0, st, d);
}
void launch_spmv_a(const DevPlan& d, hipStream_t st) {
  const dim3 grid(d.n_rblk, kRowChunk / (kThreads / 64));
  if (d.relax) hipLaunchKernelGGL(k_spmv_a<true>, grid, dim3(kThreads), 0, st, d);
  else hipLaunchKernelGGL(k_spmv_a<false>, grid, dim3(kThreads), 0, st, d);
}
void launch_trsv(const DevPlan& d, hipStream_t st) {
  switch (d.trsv_rows) {
    case 1: hipLaunchKernelGGL((k_trsv<1, 8>), dim3(d.B), dim3(kTrsvThreads), 0, st, d); break;
    case 2: hipLaunchKernelGGL((k_trsv<2, 8>), dim3(d.B), dim3(kTrsvThreads), 0, st, d); break;
    case 4: hipLaunchKernelGGL((k_trsv<4, 4>), dim3(d.B), dim3(kTrsvThreads), 0, st, d); break;
    default: hipLaunchKernelGGL((k_trsv<8, 4>), dim3(d.B), dim3(kTrsvThreads), 0, st, d); break;
  }
}
void launch_spmv_at(const DevPlan& d, hipStream_t st) {
  if (d.relax) hipLaunchKernelGGL(k_spmv_at<true>, dim3(d.n_eblk), dim3(kThreads), 0, st, d);
  else hipLaunchKernelGGL(k_spmv_at<false>, dim3(d.n_eblk), dim3(kThreads), 0, st, d);
}
void launch_scalar1(const DevPlan& d, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar1, dim3(d.B), dim3(64), 0, st, d);
}
void launch_update_e(const DevPlan& d, hipStream_t st) {
  if (d.relax) hipLaunchKernelGGL(k_update_e<true>, dim3(d.n_eblk), dim3(kThreads), 0, st, d);
  else hipLaunchKernelGGL(k_update_e<false>, dim3(d.n_eblk), dim3(kThreads), 0, st, d);
}
void launch_update_r(const DevPlan& d, hipStream_t st) {
  if (d.relax) hipLaunchKernelGGL(k_update_r<true>, dim3(d.n_rblk), dim3(kThreads), 0, st, d);
  else hipLaunchKernelGGL(k_update_r<false>, dim3(d.n_rblk), dim3(kThreads), 0, st, d);
}
void launch_scalar2(const DevPlan& d, double eps_tol, int32_t max_iter, int32_t stop, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar2, dim3(d.B), dim3(64), 0, st, d, eps_tol, max_iter, stop);
}

}  // namespace cdcs
