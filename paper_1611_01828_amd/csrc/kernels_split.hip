// The primal-only and dual-only ADMM on the decomposed pair of Section 3.1
// (the two first-order methods of the authors' earlier work that Section 5
// compares with the self-dual one: the CDCS-primal and CDCS-dual columns of
// Tables 2-4).  Both are the textbook ADMM (Boyd et al. 2011) on the
// consensus constraint between the entry vector and the clique blocks, with
// penalty rho; their step 1 is an equality-constrained least-squares step
// that reduces to the m x m matrix A D^{-1} A^T, factorised once at setup
// (D = H^T H, the number of cliques covering each entry):
//
//   primal  r = H^T(rho s + lam) - c,  (A D^-1 A^T) y = rho b - A D^-1 r,
//           x = D^-1 (r + A^T y) / rho,   s+ = Pi(H x - lam/rho),
//           lam+ = lam + rho (s+ - H x)
//   dual    r = H^T(z - lam/rho) - c,  (A D^-1 A^T) y = b / rho - A D^-1 r,
//           x = rho D^-1 (A^T y + r),  v = z - lam/rho - H x / rho,
//           z+ = Pi(v + lam/rho),      lam+ = lam + rho (v - z+)
//
// The projection Pi onto the clique PSD cones runs in the conic-step kernels
// of the self-dual method (Jacobi buckets and the tridiagonal path) through
// their stand-alone entry, the m x m solve in the self-dual method's
// triangular-solve kernel.  Buffers: x, y, q as in the self-dual plan; s (or
// z) in `s`, lam in `z`, v in `v`, r in `hsum`, D^-1 in `pinv`.  Partial
// sums have a fixed block range per instance (no atomics).
#include "device.h"

namespace cdcs {

// r = H^T(rho s + lam) - c (primal) or H^T(z - lam/rho) - c (dual), q = D^-1 r
template <bool PRIMAL>
__global__ __launch_bounds__(kThreads) void k_split_r(DevPlan d, SplitArgs a) {
  const int4 bd = d.eblk[blockIdx.x];
  if (d.st[bd.x * kNst + ST_FROZEN]) return;
  const double rho = a.rho;
  for (int e = bd.y + threadIdx.x; e < bd.z; e += kThreads) {
    double acc = 0.0;
    const int k0 = d.ent_sptr[e], k1 = d.ent_sptr[e + 1];
    for (int kb = k0; kb < k1; kb += 4) {
      int sl[4];
      double sv[4], lv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) sl[u] = d.ent_slots[min(kb + u, k1 - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sv[u] = d.s[sl[u]];
        lv[u] = d.z[sl[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (kb + u < k1) acc += PRIMAL ? rho * sv[u] + lv[u] : sv[u] - lv[u] / rho;
    }
    const double r = acc - d.c[e];
    d.hsum[e] = r;
    d.q[e] = d.pinv[e] * r;
  }
}

// g = rho b - A q (primal) or b / rho - A q (dual); one wavefront per row
template <bool PRIMAL>
__global__ __launch_bounds__(kThreads) void k_split_g(DevPlan d, SplitArgs a) {
  const int4 bd = d.rblk[blockIdx.x];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r = bd.y + blockIdx.y * (kThreads / 64) + wid;
  if (r >= bd.z || d.st[bd.x * kNst + ST_FROZEN]) return;
  constexpr int kBatch = 8;
  double acc = 0.0;
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
    for (int u = 0; u < kBatch; ++u) acc += (qb + 64 * u + lane < q1) ? av[u] * d.q[col[u]] : 0.0;
  }
  acc = wave_sum(acc);
  if (lane == 0) d.g[r] = (PRIMAL ? a.rho * d.b[r] : d.b[r] / a.rho) - acc;
}

// x = D^-1 (r + A^T y) / rho (primal) or rho D^-1 (A^T y + r) (dual); c^T x
// partial sums per entry block
template <bool PRIMAL>
__global__ __launch_bounds__(kThreads) void k_split_x(DevPlan d, SplitArgs a) {
  __shared__ double red[kThreads / 64 + 1];
  const int4 bd = d.eblk[blockIdx.x];
  if (d.st[bd.x * kNst + ST_FROZEN]) return;
  const double rho = a.rho;
  double cx = 0.0;
  for (int e = bd.y + threadIdx.x; e < bd.z; e += kThreads) {
    double atv = 0.0;
    const int q0 = d.at_ptr[e], q1 = d.at_ptr[e + 1];
    for (int qb = q0; qb < q1; qb += 4) {
      int rw[4];
      double av[4], yv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int qc = min(qb + u, q1 - 1);
        rw[u] = d.at_row[qc];
        av[u] = d.at_val[qc];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) yv[u] = d.y[rw[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (qb + u < q1) atv += av[u] * yv[u];
    }
    const double r = d.hsum[e];
    const double x = PRIMAL ? d.pinv[e] * (r + atv) / rho : (rho * d.pinv[e]) * (atv + r);
    d.x[e] = x;
    cx += d.c[e] * x;
  }
  cx = block_sum<kThreads>(cx, red);
  if (threadIdx.x == 0) d.part_e[blockIdx.x * 4 + 0] = cx;
}

// projection argument: H x - lam/rho (primal) or v + lam/rho with
// v = z - lam/rho - H x / rho (dual)
template <bool PRIMAL>
__global__ __launch_bounds__(kThreads) void k_split_w(DevPlan d, SplitArgs a) {
  const int4 bd = a.sblk[blockIdx.x];
  if (d.st[bd.x * kNst + ST_FROZEN]) return;
  const double rho = a.rho;
  for (int sl = bd.y + threadIdx.x; sl < bd.z; sl += kThreads) {
    const double hx = d.x[d.slot2ent[sl]];
    const double lam = d.z[sl];
    if (PRIMAL) {
      a.w[sl] = hx - lam / rho;
    } else {
      const double v = (d.s[sl] - lam / rho) - hx / rho;
      a.w[sl] = v + lam / rho;
    }
  }
}

// steps 2-3 after the projection p: multiplier update, the new block, and
// the residual partial sums [|p - Hx|^2 or |v - p|^2, |p|^2, |Hx|^2 or |v|^2,
// |p - old|^2, |lam+|^2]
template <bool PRIMAL>
__global__ __launch_bounds__(kThreads) void k_split_update(DevPlan d, SplitArgs a) {
  __shared__ double red[kThreads / 64 + 1];
  const int4 bd = a.sblk[blockIdx.x];
  if (d.st[bd.x * kNst + ST_FROZEN]) return;
  const double rho = a.rho;
  double t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0;
  for (int sl = bd.y + threadIdx.x; sl < bd.z; sl += kThreads) {
    const double hx = d.x[d.slot2ent[sl]];
    const double lam = d.z[sl];
    const double old = d.s[sl];
    const double p = a.p[sl];
    double ln, diff, other;
    if (PRIMAL) {
      ln = lam + rho * (p - hx);
      diff = p - hx;
      other = hx;
    } else {
      const double v = (old - lam / rho) - hx / rho;
      ln = lam + rho * (v - p);
      diff = v - p;
      other = v;
      d.v[sl] = v;
    }
    t0 += diff * diff;
    t1 += p * p;
    t2 += other * other;
    t3 += (p - old) * (p - old);
    t4 += ln * ln;
    d.s[sl] = p;
    d.z[sl] = ln;
  }
  t0 = block_sum<kThreads>(t0, red);
  t1 = block_sum<kThreads>(t1, red);
  t2 = block_sum<kThreads>(t2, red);
  t3 = block_sum<kThreads>(t3, red);
  t4 = block_sum<kThreads>(t4, red);
  if (threadIdx.x == 0) {
    double* o = a.part_s + (size_t)blockIdx.x * kSplitParts;
    o[0] = t0;
    o[1] = t1;
    o[2] = t2;
    o[3] = t3;
    o[4] = t4;
  }
}

// residuals and status (reading S3 of the oracle): eps_p = sqrt(t0) /
// max(sqrt(t1), sqrt(t2)), eps_d = rho sqrt(t3) / sqrt(t4); solved when both
// are within eps_tol; objectives c^T x and b^T y
__global__ __launch_bounds__(64) void k_split_scalar(DevPlan d, SplitArgs a, double eps_tol, int32_t max_iter,
                                                     int32_t stop) {
  const int inst = blockIdx.x;
  int32_t* st = d.st + inst * kNst;
  if (st[ST_FROZEN]) return;
  const int lane = threadIdx.x;
  double t[5] = {0, 0, 0, 0, 0}, cx = 0.0;
  for (int b = a.sblk_off[inst] + lane; b < a.sblk_off[inst + 1]; b += 64)
#pragma unroll
    for (int i = 0; i < 5; ++i) t[i] += a.part_s[(size_t)b * kSplitParts + i];
  for (int b = d.eblk_off[inst] + lane; b < d.eblk_off[inst + 1]; b += 64) cx += d.part_e[b * 4 + 0];
#pragma unroll
  for (int i = 0; i < 5; ++i) t[i] = wave_sum(t[i]);
  cx = wave_sum(cx);
  if (lane != 0) return;
  double* sc = d.sc + inst * kNsc;
  const double pden = fmax(sqrt(t[1]), sqrt(t[2]));
  const double dden = sqrt(t[4]);
  const double ep = pden > 0.0 ? sqrt(t[0]) / pden : INFINITY;
  const double ed = dden > 0.0 ? a.rho * sqrt(t[3]) / dden : INFINITY;
  const double by = sc[SC_BW];
  sc[SC_EPS_P] = ep;
  sc[SC_EPS_D] = ed;
  sc[SC_EPS_G] = fabs(cx - by) / (1.0 + fabs(cx) + fabs(by));
  sc[SC_CX] = cx;
  sc[SC_BY] = by;
  const int it = st[ST_ITER] + 1;
  st[ST_ITER] = it;
  int status = (ep <= eps_tol && ed <= eps_tol) ? 1 : 0;
  if (stop && status == 0 && it >= max_iter) status = 4;
  st[ST_STATUS] = status;
  if (stop && status != 0) st[ST_FROZEN] = 1;
}

void launch_split_r(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st) {
  if (primal) hipLaunchKernelGGL(k_split_r<true>, dim3(d.n_eblk), dim3(kThreads), 0, st, d, a);
  else hipLaunchKernelGGL(k_split_r<false>, dim3(d.n_eblk), dim3(kThreads), 0, st, d, a);
}
void launch_split_g(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st) {
  const dim3 grid(d.n_rblk, kRowChunk / (kThreads / 64));
  if (primal) hipLaunchKernelGGL(k_split_g<true>, grid, dim3(kThreads), 0, st, d, a);
  else hipLaunchKernelGGL(k_split_g<false>, grid, dim3(kThreads), 0, st, d, a);
}
void launch_split_x(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st) {
  if (primal) hipLaunchKernelGGL(k_split_x<true>, dim3(d.n_eblk), dim3(kThreads), 0, st, d, a);
  else hipLaunchKernelGGL(k_split_x<false>, dim3(d.n_eblk), dim3(kThreads), 0, st, d, a);
}
void launch_split_w(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st) {
  if (a.n_sblk <= 0) return;
  if (primal) hipLaunchKernelGGL(k_split_w<true>, dim3(a.n_sblk), dim3(kThreads), 0, st, d, a);
  else hipLaunchKernelGGL(k_split_w<false>, dim3(a.n_sblk), dim3(kThreads), 0, st, d, a);
}
void launch_split_update(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st) {
  if (a.n_sblk <= 0) return;
  if (primal) hipLaunchKernelGGL(k_split_update<true>, dim3(a.n_sblk), dim3(kThreads), 0, st, d, a);
  else hipLaunchKernelGGL(k_split_update<false>, dim3(a.n_sblk), dim3(kThreads), 0, st, d, a);
}
void launch_split_scalar(const DevPlan& d, const SplitArgs& a, double eps_tol, int32_t max_iter, int32_t stop,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_split_scalar, dim3(d.B), dim3(64), 0, st, d, a, eps_tol, max_iter, stop);
}

}  // namespace cdcs
