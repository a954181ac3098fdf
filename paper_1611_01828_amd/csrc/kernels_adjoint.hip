// Reverse-mode derivative of a solved SDP through the ADMM fixed point.
//
// With z = u - v~ the iteration (Step1)-(Step3) is z+ = T(z) =
// z + R(2 Pi(z) - z) - Pi(z), R = (I + Q)^{-1}.  At a fixed point z*, for a
// loss with g = DPi dL/du, the adjoint mu solves mu = T'^T mu + g, i.e.
//   mu <- mu - q + DPi(2 q - mu) + g,   q = (I - Q)^{-1} mu,
// and with nu = (I - Q)^{-1} mu the data gradients are
//   dL/dc = -(tau nu_x - nu_tau x),   dL/db = tau nu_y - nu_tau y.
//
// (I - Q) q = mu is solved with the same cached factor as step 1:
//   t   = mu_x - A^T mu_y - H^T(mu_v - mu_s)/2
//   a   = F^{-1} t  (F = I + D/2 + A^T A, matrix inversion lemma:
//         p = P^{-1} t, w = K^{-1} A p, a = p - P^{-1} A^T w, and A a = w)
//   q_tau = (mu_tau + b^T mu_y - e^T a) / (1 + ||b||^2 + e^T phi),
//           e = c - A^T b, phi = F^{-1}(c + A^T b)
//   q_x = a + q_tau phi,  q_y = mu_y + w + q_tau A phi - b q_tau,
//   q_s = (mu_s + mu_v + H q_x)/2,  q_v = (mu_v - mu_s + H q_x)/2.
// DPi on a PSD block at Y = V diag(lam) V^T maps dY to V (B o (V^T dY V)) V^T
// (Daleckii-Krein divided differences B).  Free blocks pass through; the tau
// block passes iff tau > 0.
#include "cone_common.h"

namespace cdcs {

// per-instance adjoint scalars (double as[B * kNas])
enum As { AS_QT = 0, AS_GT, AS_DEN2, AS_DIFF2, AS_NORM2, AS_BY, AS_EA, kNas = 8 };

struct AdjPlan {
  DevPlan d;                 // forward data (state at the solution is read only)
  double* as;                // B * kNas
  double* mu_x;
  double* mu_s;
  double* mu_y;
  double* mu_v;
  double* mu_t;              // B
  double* qx;                // NE
  const double* gx;          // NE: dL/dx = w / tau
  const double* phi;         // NE
  const double* ev;          // NE: c - A^T b
  const double* aphi;        // M: A phi
  const double* eig;         // cached eigenpairs per clique
  const int64_t* eig_off;    // P
  double* dc;                // NE output
  double* db;                // M output
};

// 1. eigenpairs of the s-block of z* = u* - v~* (Y = smat(s - z)) per clique
template <int KMAX, int NT>
__global__ __launch_bounds__(NT) void k_adj_eig(AdjPlan ap, const int32_t* tasks) {
  __shared__ double A[KMAX * KMAX];
  __shared__ double V[KMAX * KMAX];
  __shared__ JacRot<KMAX, double> rot;
  __shared__ double red[NT / 64 + 1];
  const DevPlan& d = ap.d;
  const int k = tasks[blockIdx.x];
  const int K = d.clq_size[k];
  const int KP = K + (K & 1);
  const int64_t s0 = d.clq_slot[k];
  for (int idx = threadIdx.x; idx < KP * KP; idx += NT) {
    const int i = idx / KP, j = idx - (idx / KP) * KP;
    double yv = 0.0;
    if (i < K && j < K) {
      const int a = i > j ? i : j, bq = i > j ? j : i;
      const int64_t sl = s0 + packed_index(a, bq, K);
      yv = d.s[sl] - d.z[sl];
      if (a != bq) yv *= kInvSqrt2;
    }
    A[i * KMAX + j] = yv;
    V[i * KMAX + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_lds<KMAX, NT>(A, V, K, KP, rot, red);
  double* out = const_cast<double*>(ap.eig) + ap.eig_off[k];
  for (int idx = threadIdx.x; idx < K * K; idx += NT) {
    const int i = idx / K, l = idx - (idx / K) * K;
    out[idx] = V[i * KMAX + l];                 // out[i*K + l] = V_il (eigenvector l)
  }
  for (int l = threadIdx.x; l < K; l += NT) out[K * K + l] = A[l * KMAX + l];
}

// A^T u at the 64 entries of sliced-ELL chunk ch (one per lane; see k_spmv_at)
__device__ __forceinline__ double at_chunk_dot(const DevPlan& d, int ch, int lane, const double* u) {
  const int len = d.at_chlen[ch];
  const int32_t* srow = d.at_srow + d.at_chptr[ch] + lane;
  const double* sval = d.at_sval + d.at_chptr[ch] + lane;
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < len; ++k) acc += sval[(size_t)k * 64] * u[srow[(size_t)k * 64]];
  return acc;
}

// 2. t and p = P^{-1} t
__global__ __launch_bounds__(kThreads) void k_adj_rhs(AdjPlan ap) {
  const DevPlan& d = ap.d;
  const int4 bd = d.eblk[blockIdx.x];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nch = (bd.z - bd.y + 63) >> 6;
  for (int c = wid; c < nch; c += kThreads / 64) {
    const int ch = d.at_choff[blockIdx.x] + c;
    const int e = d.at_sent[(size_t)ch * 64 + lane];
    const double aty = at_chunk_dot(d, ch, lane, ap.mu_y);
    if (e < 0) continue;
    double hs = 0.0;
    for (int k = d.ent_sptr[e]; k < d.ent_sptr[e + 1]; ++k) {
      const int sl = d.ent_slots[k];
      hs += ap.mu_v[sl] - ap.mu_s[sl];
    }
    const double t = ap.mu_x[e] - aty - 0.5 * hs;
    d.q[e] = d.pinv[e] * t;
  }
}

// 3. g = A p ; partial b^T mu_y
__global__ __launch_bounds__(kThreads) void k_adj_ap(AdjPlan ap) {
  __shared__ double red[kThreads / 64 + 1];
  const DevPlan& d = ap.d;
  const int4 bd = d.rblk[blockIdx.x];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int r = bd.y + wid; r < bd.z; r += kThreads / 64) {
    // batches of 8 clamped loads per lane in flight (as in k_spmv_a)
    double acc = 0.0;
    const int q0 = d.a_ptr[r], q1 = d.a_ptr[r + 1];
    for (int qb = q0; qb < q1; qb += 64 * 8) {
      int col[8];
      double av[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int qc = min(qb + 64 * u + lane, q1 - 1);
        col[u] = d.a_col[qc];
        av[u] = d.a_val[qc];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += ((qb + 64 * u + lane < q1) ? av[u] : 0.0) * d.q[col[u]];
    }
    acc = wave_sum(acc);
    if (lane == 0) d.g[r] = acc;
  }
  double by = 0.0;
  for (int r = bd.y + threadIdx.x; r < bd.z; r += kThreads) by += d.b[r] * ap.mu_y[r];
  by = block_sum<kThreads>(by, red);
  if (threadIdx.x == 0) d.part_r[blockIdx.x * 4 + 3] = by;
}

// 5. a = p - P^{-1} A^T w ; partial e^T a
__global__ __launch_bounds__(kThreads) void k_adj_a(AdjPlan ap) {
  __shared__ double red[kThreads / 64 + 1];
  const DevPlan& d = ap.d;
  const int4 bd = d.eblk[blockIdx.x];
  double ea = 0.0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nch = (bd.z - bd.y + 63) >> 6;
  for (int c = wid; c < nch; c += kThreads / 64) {
    const int ch = d.at_choff[blockIdx.x] + c;
    const int e = d.at_sent[(size_t)ch * 64 + lane];
    const double acc = at_chunk_dot(d, ch, lane, d.w);
    if (e < 0) continue;
    const double a = d.q[e] - d.pinv[e] * acc;
    d.px[e] = a;
    ea += ap.ev[e] * a;
  }
  ea = block_sum<kThreads>(ea, red);
  if (threadIdx.x == 0) d.part_e[blockIdx.x * 4 + 0] = ea;
}

// 6. q_tau
__global__ __launch_bounds__(64) void k_adj_s1(AdjPlan ap) {
  const DevPlan& d = ap.d;
  const int inst = blockIdx.x;
  double ea = 0.0, by = 0.0;
  for (int b = d.eblk_off[inst] + threadIdx.x; b < d.eblk_off[inst + 1]; b += 64) ea += d.part_e[b * 4 + 0];
  for (int b = d.rblk_off[inst] + threadIdx.x; b < d.rblk_off[inst + 1]; b += 64) by += d.part_r[b * 4 + 3];
  ea = wave_sum(ea);
  by = wave_sum(by);
  if (threadIdx.x == 0) {
    double* as = ap.as + inst * kNas;
    as[AS_EA] = ea;
    as[AS_BY] = by;
    as[AS_QT] = (ap.mu_t[inst] + by - ea) / as[AS_DEN2];
  }
}

// 7. q_x and the x block of mu (final = 1: dL/dc instead)
__global__ __launch_bounds__(kThreads) void k_adj_ue(AdjPlan ap, int final_pass, int use_g) {
  __shared__ double red[kThreads / 64 + 1];
  const DevPlan& d = ap.d;
  const int4 bd = d.eblk[blockIdx.x];
  const int inst = bd.x;
  const double qt = ap.as[inst * kNas + AS_QT];
  const double tau = d.sc[inst * kNsc + SC_TAU];
  double df = 0.0, nm = 0.0;
  for (int e = bd.y + threadIdx.x; e < bd.z; e += kThreads) {
    const double qx = d.px[e] + qt * ap.phi[e];
    if (final_pass) {
      ap.dc[e] = -(tau * qx - qt * d.x[e]);
    } else {
      ap.qx[e] = qx;
      const double mn = qx + (use_g ? ap.gx[e] : 0.0);
      const double dd = mn - ap.mu_x[e];
      ap.mu_x[e] = mn;
      df += dd * dd;
      nm += mn * mn;
    }
  }
  if (final_pass) return;
  df = block_sum<kThreads>(df, red);
  nm = block_sum<kThreads>(nm, red);
  if (threadIdx.x == 0) {
    d.part_e[blockIdx.x * 4 + 1] = df;
    d.part_e[blockIdx.x * 4 + 2] = nm;
  }
}

// 8. q_y and the y block of mu (final = 1: dL/db instead)
__global__ __launch_bounds__(kThreads) void k_adj_ur(AdjPlan ap, int final_pass) {
  __shared__ double red[kThreads / 64 + 1];
  const DevPlan& d = ap.d;
  const int4 bd = d.rblk[blockIdx.x];
  const int inst = bd.x;
  const double qt = ap.as[inst * kNas + AS_QT];
  const double tau = d.sc[inst * kNsc + SC_TAU];
  double df = 0.0, nm = 0.0;
  for (int r = bd.y + threadIdx.x; r < bd.z; r += kThreads) {
    const double qy = ap.mu_y[r] + d.w[r] + qt * ap.aphi[r] - d.b[r] * qt;
    if (final_pass) {
      ap.db[r] = tau * qy - qt * d.y[r];
    } else {
      const double dd = qy - ap.mu_y[r];
      ap.mu_y[r] = qy;
      df += dd * dd;
      nm += qy * qy;
    }
  }
  if (final_pass) return;
  df = block_sum<kThreads>(df, red);
  nm = block_sum<kThreads>(nm, red);
  if (threadIdx.x == 0) {
    d.part_r[blockIdx.x * 4 + 1] = df;
    d.part_r[blockIdx.x * 4 + 2] = nm;
  }
}

// 9. s and v blocks of mu: q_s, q_v from H q_x, then DPi on the clique block
template <int KMAX, int NT>
__global__ __launch_bounds__(NT) void k_adj_cone(AdjPlan ap, const int32_t* tasks) {
  // V and one K x K work matrix in LDS (two arrays: 147 KB at KMAX = 96);
  // each product's entries are formed in registers (NO per thread) and
  // written over the work matrix after a barrier
  constexpr int NO = (KMAX * KMAX + NT - 1) / NT;
  __shared__ double Vs[KMAX * KMAX];
  __shared__ double M[KMAX * KMAX];
  __shared__ double lam[KMAX];
  __shared__ double red[NT / 64 + 1];
  const DevPlan& d = ap.d;
  const int k = tasks[blockIdx.x];
  const int K = d.clq_size[k];
  const int KK = K * K;
  const int64_t s0 = d.clq_slot[k];
  const double* eg = ap.eig + ap.eig_off[k];
  const int tid = threadIdx.x;
  const int nslot = K * (K + 1) / 2;
  for (int idx = tid; idx < KK; idx += NT) Vs[idx] = eg[idx];
  for (int l = tid; l < K; l += NT) lam[l] = eg[KK + l];
  // D = smat(2 q_s - mu_s) into M (full symmetric)
  for (int t = tid; t < nslot; t += NT) {
    int a, bq;
    unpack_index(t, K, a, bq);
    const int64_t sl = s0 + t;
    const double hq = ap.qx[d.slot2ent[sl]];
    const double qs = 0.5 * (ap.mu_s[sl] + ap.mu_v[sl] + hq);
    double dv = 2.0 * qs - ap.mu_s[sl];
    if (a != bq) dv *= kInvSqrt2;
    M[a * K + bq] = dv;
    M[bq * K + a] = dv;
  }
  __syncthreads();
  double r[NO];
  // T = D V
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int idx = tid + u * NT;
    double acc = 0.0;
    if (idx < KK) {
      const int i = idx / K, l = idx - (idx / K) * K;
      for (int j = 0; j < K; ++j) acc += M[i * K + j] * Vs[j * K + l];
    }
    r[u] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NO; ++u)
    if (tid + u * NT < KK) M[tid + u * NT] = r[u];
  __syncthreads();
  // B o (V^T T), B the divided differences of max(lambda, 0)
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int idx = tid + u * NT;
    double acc = 0.0;
    if (idx < KK) {
      const int p = idx / K, l = idx - (idx / K) * K;
      for (int i = 0; i < K; ++i) acc += Vs[i * K + p] * M[i * K + l];
      const double lp = lam[p], ll = lam[l];
      double bw;
      if (lp > 0.0 && ll > 0.0) bw = 1.0;
      else if (lp <= 0.0 && ll <= 0.0) bw = 0.0;
      else bw = (fmax(lp, 0.0) - fmax(ll, 0.0)) / (lp - ll);
      acc *= bw;
    }
    r[u] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NO; ++u)
    if (tid + u * NT < KK) M[tid + u * NT] = r[u];
  __syncthreads();
  // T = (B o ...) V^T
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int idx = tid + u * NT;
    double acc = 0.0;
    if (idx < KK) {
      const int p = idx / K, j = idx - (idx / K) * K;
      for (int l = 0; l < K; ++l) acc += M[p * K + l] * Vs[j * K + l];
    }
    r[u] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NO; ++u)
    if (tid + u * NT < KK) M[tid + u * NT] = r[u];
  __syncthreads();
  // result = V T on the packed slots, and the adjoint update of mu_s, mu_v
  double df = 0.0, nm = 0.0;
  for (int t = tid; t < nslot; t += NT) {
    int a, bq;
    unpack_index(t, K, a, bq);
    double rr = 0.0;
    for (int p = 0; p < K; ++p) rr += Vs[a * K + p] * M[p * K + bq];
    if (a != bq) rr *= kSqrt2;
    const int64_t sl = s0 + t;
    const double hq = ap.qx[d.slot2ent[sl]];
    const double ms = ap.mu_s[sl], mv = ap.mu_v[sl];
    const double qs = 0.5 * (ms + mv + hq);
    const double qv = 0.5 * (mv - ms + hq);
    const double ns = ms - qs + rr;
    ap.mu_s[sl] = ns;
    ap.mu_v[sl] = qv;
    df += (ns - ms) * (ns - ms) + (qv - mv) * (qv - mv);
    nm += ns * ns + qv * qv;
  }
  df = block_sum<NT>(df, red);
  nm = block_sum<NT>(nm, red);
  if (tid == 0) {
    d.part_c[2 * k] = df;
    d.part_c[2 * k + 1] = nm;
  }
}

// 10. tau block of mu and the convergence measures
__global__ __launch_bounds__(64) void k_adj_s2(AdjPlan ap, int use_g) {
  const DevPlan& d = ap.d;
  const int inst = blockIdx.x;
  double df = 0.0, nm = 0.0;
  for (int b = d.eblk_off[inst] + threadIdx.x; b < d.eblk_off[inst + 1]; b += 64) {
    df += d.part_e[b * 4 + 1];
    nm += d.part_e[b * 4 + 2];
  }
  for (int b = d.rblk_off[inst] + threadIdx.x; b < d.rblk_off[inst + 1]; b += 64) {
    df += d.part_r[b * 4 + 1];
    nm += d.part_r[b * 4 + 2];
  }
  for (int k = d.clq_off[inst] + threadIdx.x; k < d.clq_off[inst + 1]; k += 64) {
    df += d.part_c[2 * k];
    nm += d.part_c[2 * k + 1];
  }
  df = wave_sum(df);
  nm = wave_sum(nm);
  if (threadIdx.x == 0) {
    double* as = ap.as + inst * kNas;
    const double qt = as[AS_QT], gt = use_g ? as[AS_GT] : 0.0, mt = ap.mu_t[inst];
    const double tau = d.sc[inst * kNsc + SC_TAU];
    const double mn = (tau > 0.0) ? qt + gt : mt - qt + gt;
    ap.mu_t[inst] = mn;
    as[AS_DIFF2] = df + (mn - mt) * (mn - mt);
    as[AS_NORM2] = nm + mn * mn;
  }
}

// ---------------------------------------------------------------------------
// Batched restarted GMRES on (I - T'^T) mu = g.  Vectors are flat:
// [x (NE) | s (NS) | y (M) | v (NS) | tau (B)]; seg[10 i .. 10 i + 9] holds
// the five [lo, hi) ranges of instance i, inst_of maps an element to its
// instance.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_seg_dots(const double* w, const double* Vb, int64_t NF,
                                                  const int64_t* seg, double* out, int B) {
  __shared__ double red[256 / 64 + 1];
  const int i = blockIdx.x, k = blockIdx.y;
  const double* v = Vb + (size_t)k * NF;
  double acc = 0.0;
  for (int q = 0; q < 5; ++q) {
    const int64_t lo = seg[10 * i + 2 * q], hi = seg[10 * i + 2 * q + 1];
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) acc += w[e] * v[e];
  }
  acc = block_sum<256>(acc, red);
  if (threadIdx.x == 0) out[k * B + i] = acc;
}

// w += sign * sum_k coef[k, inst(e)] V_k
__global__ __launch_bounds__(256) void k_flat_axpy_multi(double* w, const double* Vb, int64_t NF, int nk,
                                                         const double* coef, const int32_t* inst_of, int B,
                                                         double sign) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= NF) return;
  const int i = inst_of[e];
  double acc = 0.0;
  for (int k = 0; k < nk; ++k) acc += coef[k * B + i] * Vb[(size_t)k * NF + e];
  w[e] += sign * acc;
}

__global__ __launch_bounds__(256) void k_flat_scale(double* out, const double* w, const double* sc,
                                                    const int32_t* inst_of, int64_t NF) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < NF) out[e] = w[e] * sc[inst_of[e]];
}

// out = a - b
__global__ __launch_bounds__(256) void k_flat_sub(double* out, const double* a, const double* b, int64_t NF) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < NF) out[e] = a[e] - b[e];
}


// start of a cycle: beta = ||g - A mu|| (nrm holds its square); an instance
// stops when beta <= tol ||g|| or when beta fell by less than 10 % over the
// last kGmWindow restarts
__global__ void k_gm_begin(GmState g, const double* nrm, double* scale, int B, int R, double tol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const double beta = sqrt(nrm[i]);
  int done = g.done[i];
  if (!done) {
    const int nh = g.nhist[i];
    if (beta <= tol * fmax(g.gnorm[i], 1e-300) ||
        (nh >= kGmWindow && beta > kGmStall * g.hist[(size_t)i * kGmWindow + nh % kGmWindow]))
      done = 1;
    g.hist[(size_t)i * kGmWindow + nh % kGmWindow] = beta;
    g.nhist[i] = nh + 1;
    g.done[i] = done;
  }
  g.gam[(size_t)i * (R + 1)] = beta;
  scale[i] = beta > 0.0 ? 1.0 / beta : 0.0;
  g.jlim[i] = done ? 0 : -1;
  if (!done) g.alldone[0] = 0;   // (set to 1 by the host before the launch)
}

// Krylov step j: Hessenberg column from the two Gram-Schmidt passes (d1, d2:
// (j+1) x B) and the new norm, previous rotations, a new one, gamma, the
// instance's stopping column, and the scale of the next basis vector
__global__ void k_gm_step(GmState g, const double* d1, const double* d2, const double* nrm, double* scale, int B,
                          int R, int j, double tol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  double* Hc = g.H + ((size_t)i * (R + 1)) * R + (size_t)j * (R + 1);
  for (int k = 0; k <= j; ++k) Hc[k] = d1[(size_t)k * B + i] + d2[(size_t)k * B + i];
  const double hn = sqrt(nrm[i]);
  Hc[j + 1] = hn;
  scale[i] = hn > 1e-300 ? 1.0 / hn : 0.0;
  double* c_ = g.cs + (size_t)i * R;
  double* s_ = g.sn + (size_t)i * R;
  for (int k = 0; k < j; ++k) {
    const double h0 = Hc[k], h1 = Hc[k + 1];
    Hc[k] = c_[k] * h0 + s_[k] * h1;
    Hc[k + 1] = -s_[k] * h0 + c_[k] * h1;
  }
  const double h0 = Hc[j], h1 = Hc[j + 1];
  const double r = hypot(h0, h1);
  c_[j] = r > 0.0 ? h0 / r : 1.0;
  s_[j] = r > 0.0 ? h1 / r : 0.0;
  Hc[j] = r;
  Hc[j + 1] = 0.0;
  double* gi = g.gam + (size_t)i * (R + 1);
  gi[j + 1] = -s_[j] * gi[j];
  gi[j] = c_[j] * gi[j];
  if (g.jlim[i] < 0 && fabs(gi[j + 1]) <= tol * fmax(g.gnorm[i], 1e-300)) g.jlim[i] = j + 1;
}

// end of a cycle of jdone steps: y from H y = gamma over the instance's
// columns (back substitution), coef[k B + i] = y_k (zero past them)
__global__ void k_gm_solve(GmState g, double* coef, int B, int R, int jdone) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const int ji = g.jlim[i] < 0 ? jdone : g.jlim[i];
  const double* Hm = g.H + ((size_t)i * (R + 1)) * R;
  const double* gi = g.gam + (size_t)i * (R + 1);
  double y[32];
  for (int k = ji - 1; k >= 0; --k) {
    double t = gi[k];
    for (int l = k + 1; l < ji; ++l) t -= Hm[(size_t)l * (R + 1) + k] * y[l];
    const double dkk = Hm[(size_t)k * (R + 1) + k];
    y[k] = dkk != 0.0 ? t / dkk : 0.0;
  }
  for (int k = 0; k < jdone; ++k) coef[(size_t)k * B + i] = k < ji ? y[k] : 0.0;
}

// final relative residual and reason per instance (0 within tol, 1 stalled,
// 2 iteration limit)
__global__ void k_gm_final(GmState g, const double* nrm, double* resid, int32_t* reason, int B, double tol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const double gn = g.gnorm[i];
  const double rel = gn > 0.0 ? sqrt(nrm[i]) / gn : 0.0;
  resid[i] = rel;
  reason[i] = rel <= tol ? 0 : (g.done[i] ? 1 : 2);
}

void launch_gm_begin(const GmState& g, const double* nrm, double* scale, int B, int R, double tol,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_gm_begin, dim3((B + 63) / 64), dim3(64), 0, st, g, nrm, scale, B, R, tol);
}
void launch_gm_step(const GmState& g, const double* d1, const double* d2, const double* nrm, double* scale, int B,
                    int R, int j, double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_step, dim3((B + 63) / 64), dim3(64), 0, st, g, d1, d2, nrm, scale, B, R, j, tol);
}
void launch_gm_solve(const GmState& g, double* coef, int B, int R, int jdone, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_solve, dim3((B + 63) / 64), dim3(64), 0, st, g, coef, B, R, jdone);
}
void launch_gm_final(const GmState& g, const double* nrm, double* resid, int32_t* reason, int B, double tol,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_gm_final, dim3((B + 63) / 64), dim3(64), 0, st, g, nrm, resid, reason, B, tol);
}

void launch_seg_dots(const double* w, const double* Vb, int64_t NF, int nk, const int64_t* seg, double* out,
                     int B, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_dots, dim3(B, nk), dim3(256), 0, st, w, Vb, NF, seg, out, B);
}
void launch_flat_axpy_multi(double* w, const double* Vb, int64_t NF, int nk, const double* coef,
                            const int32_t* inst_of, int B, double sign, hipStream_t st) {
  hipLaunchKernelGGL(k_flat_axpy_multi, dim3((NF + 255) / 256), dim3(256), 0, st, w, Vb, NF, nk, coef, inst_of, B,
                     sign);
}
void launch_flat_scale(double* out, const double* w, const double* sc, const int32_t* inst_of, int64_t NF,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_flat_scale, dim3((NF + 255) / 256), dim3(256), 0, st, out, w, sc, inst_of, NF);
}
__global__ __launch_bounds__(256) void k_flat_sqrt(double* out, const double* a, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) out[e] = sqrt(a[e]);
}
void launch_flat_sqrt(double* out, const double* a, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_flat_sqrt, dim3((n + 255) / 256), dim3(256), 0, st, out, a, n);
}
void launch_flat_sub(double* out, const double* a, const double* b, int64_t NF, hipStream_t st) {
  hipLaunchKernelGGL(k_flat_sub, dim3((NF + 255) / 256), dim3(256), 0, st, out, a, b, NF);
}

void launch_adj_eig(const AdjPlan& ap, const int32_t* tasks, int32_t ntask, int kmax, hipStream_t st);
void launch_adj_iteration(const AdjPlan& ap, const int32_t* const* tasks, const int32_t* ntasks,
                          int final_pass, int use_g, hipStream_t st);

void launch_adj_eig(const AdjPlan& ap, const int32_t* tasks, int32_t ntask, int kmax, hipStream_t st) {
  if (ntask <= 0) return;
  if (kmax <= 16) hipLaunchKernelGGL((k_adj_eig<16, 64>), dim3(ntask), dim3(64), 0, st, ap, tasks);
  else if (kmax <= 32) hipLaunchKernelGGL((k_adj_eig<32, 128>), dim3(ntask), dim3(128), 0, st, ap, tasks);
  else if (kmax <= 64) hipLaunchKernelGGL((k_adj_eig<64, 256>), dim3(ntask), dim3(256), 0, st, ap, tasks);
  else hipLaunchKernelGGL((k_adj_eig<96, 512>), dim3(ntask), dim3(512), 0, st, ap, tasks);
}

// tasks[0..3]: clique lists for K <= 16, <= 32, <= 64, <= 96
void launch_adj_iteration(const AdjPlan& ap, const int32_t* const* tasks, const int32_t* ntasks,
                          int final_pass, int use_g, hipStream_t st) {
  const DevPlan& d = ap.d;
  hipLaunchKernelGGL(k_adj_rhs, dim3(d.n_eblk), dim3(kThreads), 0, st, ap);
  hipLaunchKernelGGL(k_adj_ap, dim3(d.n_rblk), dim3(kThreads), 0, st, ap);
  launch_trsv(d, st);
  hipLaunchKernelGGL(k_adj_a, dim3(d.n_eblk), dim3(kThreads), 0, st, ap);
  hipLaunchKernelGGL(k_adj_s1, dim3(d.B), dim3(64), 0, st, ap);
  hipLaunchKernelGGL(k_adj_ue, dim3(d.n_eblk), dim3(kThreads), 0, st, ap, final_pass, use_g);
  hipLaunchKernelGGL(k_adj_ur, dim3(d.n_rblk), dim3(kThreads), 0, st, ap, final_pass);
  if (final_pass) return;
  if (ntasks[0]) hipLaunchKernelGGL((k_adj_cone<16, 64>), dim3(ntasks[0]), dim3(64), 0, st, ap, tasks[0]);
  if (ntasks[1]) hipLaunchKernelGGL((k_adj_cone<32, 128>), dim3(ntasks[1]), dim3(128), 0, st, ap, tasks[1]);
  if (ntasks[2]) hipLaunchKernelGGL((k_adj_cone<64, 256>), dim3(ntasks[2]), dim3(256), 0, st, ap, tasks[2]);
  if (ntasks[3]) hipLaunchKernelGGL((k_adj_cone<96, 512>), dim3(ntasks[3]), dim3(512), 0, st, ap, tasks[3]);
  hipLaunchKernelGGL(k_adj_s2, dim3(d.B), dim3(64), 0, st, ap, use_g);
}

}  // namespace cdcs
