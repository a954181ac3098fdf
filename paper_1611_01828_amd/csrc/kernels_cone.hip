// Conic step (eq. Step2, PSD part) fused with the dual update (eq. Step3)
// for cliques of up to 96 vertices: one workgroup per clique, the block held
// in LDS and diagonalised by cyclic two-sided Jacobi (Jacobi 1846; the
// symmetric 2x2 Schur rotation and round-robin parallel ordering of Golub &
// Van Loan, Matrix Computations, Sections 8.5.2-8.5.5).
//
// Per clique k (svec blocks, H_k a 0/1 gather):
//   Y   = u_s - z = (s - z - v + H_k x+) / 2
//   v+  = (s + z + v - H_k x+) / 2
//   s+  = Pi_+(Y) = V max(Lambda, 0) V^T
//   z+  = z - u_s + s+ = s+ - Y
// plus the partial sums ||H_k x+ - s+||^2 and ||v+ - z+||^2 for the residuals.
#include "cone_common.h"

namespace cdcs {

template <int KMAX, int NT>
__global__ __launch_bounds__(NT) void k_cone_jacobi(DevPlan d, const int32_t* tasks) {
  __shared__ double A[KMAX * KMAX];
  __shared__ double V[KMAX * KMAX];
  __shared__ double rc[KMAX / 2], rs[KMAX / 2], rt[KMAX / 2];
  __shared__ int rp[KMAX / 2], rq[KMAX / 2];
  __shared__ int sel[KMAX];
  __shared__ int meta[2];
  __shared__ double red[NT / 64 + 1];
  const int k = tasks[blockIdx.x];
  const int inst = d.clq_inst[k];
  if (d.st[inst * kNst + ST_FROZEN]) return;
  const int K = d.clq_size[k];
  const int KP = K + (K & 1);
  const int64_t s0 = d.clq_slot[k];
  const int tid = threadIdx.x;
  // gather Y = smat((s - z - v + H_k x+) / 2); V = I
  for (int idx = tid; idx < KP * KP; idx += NT) {
    const int i = idx / KP, j = idx - (idx / KP) * KP;
    double yv = 0.0;
    if (i < K && j < K) {
      const int a = i > j ? i : j, bq = i > j ? j : i;
      const int64_t sl = s0 + packed_index(a, bq, K);
      const double xv = d.x[d.slot2ent[sl]];
      yv = 0.5 * (d.s[sl] - d.z[sl] - d.v[sl] + xv);
      if (a != bq) yv *= kInvSqrt2;
    }
    A[i * KMAX + j] = yv;
    V[i * KMAX + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_lds<KMAX, NT>(A, V, K, KP, rc, rs, rt, rp, rq, red);
  choose_side<NT>(A, K, KMAX, sel, meta);
  const int nsel = meta[0], pos = meta[1];
  // epilogue over packed slots
  const int nslot = K * (K + 1) / 2;
  double ex = 0.0, ev = 0.0;
  for (int t = tid; t < nslot; t += NT) {
    int a, bq;
    unpack_index(t, K, a, bq);
    double acc = 0.0;
    for (int u = 0; u < nsel; ++u) {
      const int l = sel[u];
      acc += V[a * KMAX + l] * A[l * KMAX + l] * V[bq * KMAX + l];
    }
    const int64_t sl = s0 + t;
    const double sv = d.s[sl], zv = d.z[sl], vv = d.v[sl];
    const double xv = d.x[d.slot2ent[sl]];
    const double yvec = 0.5 * (sv - zv - vv + xv);          // svec(Y) entry
    const double sc = (a == bq) ? 1.0 : kSqrt2;
    const double sp = pos ? acc * sc : yvec - acc * sc;      // svec(Pi_+(Y))
    const double zn = sp - yvec;
    const double vn = 0.5 * (sv + zv + vv - xv);
    d.s[sl] = sp;
    d.z[sl] = zn;
    d.v[sl] = vn;
    ex += (xv - sp) * (xv - sp);
    ev += (vn - zn) * (vn - zn);
  }
  ex = block_sum<NT>(ex, red);
  ev = block_sum<NT>(ev, red);
  if (tid == 0) {
    d.part_c[k * 2 + 0] = ex;
    d.part_c[k * 2 + 1] = ev;
  }
}

// Stand-alone projection of packed blocks: out_k = svec(Pi_+(smat(in_k))).
template <int KMAX, int NT>
__global__ __launch_bounds__(NT) void k_psd_jacobi(const int32_t* sizes, const int64_t* offs,
                                                   const int32_t* tasks, const double* in,
                                                   double* out) {
  __shared__ double A[KMAX * KMAX];
  __shared__ double V[KMAX * KMAX];
  __shared__ double rc[KMAX / 2], rs[KMAX / 2], rt[KMAX / 2];
  __shared__ int rp[KMAX / 2], rq[KMAX / 2];
  __shared__ int sel[KMAX];
  __shared__ int meta[2];
  __shared__ double red[NT / 64 + 1];
  const int k = tasks[blockIdx.x];
  const int K = sizes[k];
  const int KP = K + (K & 1);
  const int64_t o = offs[k];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < KP * KP; idx += NT) {
    const int i = idx / KP, j = idx - (idx / KP) * KP;
    double yv = 0.0;
    if (i < K && j < K) {
      const int a = i > j ? i : j, bq = i > j ? j : i;
      yv = in[o + packed_index(a, bq, K)];
      if (a != bq) yv *= kInvSqrt2;
    }
    A[i * KMAX + j] = yv;
    V[i * KMAX + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_lds<KMAX, NT>(A, V, K, KP, rc, rs, rt, rp, rq, red);
  choose_side<NT>(A, K, KMAX, sel, meta);
  const int nsel = meta[0], pos = meta[1];
  const int nslot = K * (K + 1) / 2;
  for (int t = tid; t < nslot; t += NT) {
    int a, bq;
    unpack_index(t, K, a, bq);
    double acc = 0.0;
    for (int u = 0; u < nsel; ++u) {
      const int l = sel[u];
      acc += V[a * KMAX + l] * A[l * KMAX + l] * V[bq * KMAX + l];
    }
    const double sc = (a == bq) ? 1.0 : kSqrt2;
    const double yvec = in[o + t];
    out[o + t] = pos ? acc * sc : yvec - acc * sc;   // each element read, then written, by one thread
  }
}

void launch_cone_jacobi(const DevPlan& d, const int32_t* tasks, int32_t ntask, int kmax, hipStream_t st) {
  if (ntask <= 0) return;
  if (kmax <= 16)
    hipLaunchKernelGGL((k_cone_jacobi<16, 64>), dim3(ntask), dim3(64), 0, st, d, tasks);
  else if (kmax <= 32)
    hipLaunchKernelGGL((k_cone_jacobi<32, 128>), dim3(ntask), dim3(128), 0, st, d, tasks);
  else if (kmax <= 64)
    hipLaunchKernelGGL((k_cone_jacobi<64, 256>), dim3(ntask), dim3(256), 0, st, d, tasks);
  else
    hipLaunchKernelGGL((k_cone_jacobi<96, 512>), dim3(ntask), dim3(512), 0, st, d, tasks);
}

void launch_psd_project(const int32_t* sizes, const int64_t* offs, const int32_t* tasks, int32_t ntask,
                        int kmax, const double* in, double* out, hipStream_t st) {
  if (ntask <= 0) return;
  if (kmax <= 16)
    hipLaunchKernelGGL((k_psd_jacobi<16, 64>), dim3(ntask), dim3(64), 0, st, sizes, offs, tasks, in, out);
  else if (kmax <= 32)
    hipLaunchKernelGGL((k_psd_jacobi<32, 128>), dim3(ntask), dim3(128), 0, st, sizes, offs, tasks, in, out);
  else if (kmax <= 64)
    hipLaunchKernelGGL((k_psd_jacobi<64, 256>), dim3(ntask), dim3(256), 0, st, sizes, offs, tasks, in, out);
  else
    hipLaunchKernelGGL((k_psd_jacobi<96, 512>), dim3(ntask), dim3(512), 0, st, sizes, offs, tasks, in, out);
}

}  // namespace cdcs
