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
#include "device.h"

namespace cdcs {

namespace {

constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kInvSqrt2 = 0.70710678118654752;

// packed column-major lower index of (a, b), a >= b, in a K x K block
__device__ __forceinline__ int packed_index(int a, int b, int K) {
  return b * K - (b * (b - 1)) / 2 + (a - b);
}

// inverse of packed_index: column b is the largest with b K - b (b-1)/2 <= t
__device__ __forceinline__ void unpack_index(int t, int K, int& a, int& b) {
  const double k2 = 2.0 * K + 1.0;
  int bb = (int)((k2 - sqrt(k2 * k2 - 8.0 * t)) * 0.5);
  if (bb < 0) bb = 0;
  if (bb > K - 1) bb = K - 1;
  while (bb > 0 && packed_index(bb, bb, K) > t) --bb;
  while (bb < K - 1 && packed_index(bb + 1, bb + 1, K) <= t) ++bb;
  b = bb;
  a = bb + (t - packed_index(bb, bb, K));
}

// Symmetric Schur 2x2: (c, s, t) with t = tan(theta) annihilating A_pq.
__device__ __forceinline__ void schur2(double app, double aqq, double apq, double& c, double& s,
                                      double& t) {
  if (apq == 0.0) {
    c = 1.0;
    s = 0.0;
    t = 0.0;
    return;
  }
  const double theta = (aqq - app) / (2.0 * apq);
  const double at = fabs(theta);
  double tt;
  if (at > 1e150) {
    tt = 0.5 / theta;
  } else {
    tt = 1.0 / (at + sqrt(1.0 + at * at));
    if (theta < 0.0) tt = -tt;
  }
  c = 1.0 / sqrt(1.0 + tt * tt);
  s = tt * c;
  t = tt;
}

}  // namespace

// Cyclic Jacobi on the KP x KP (KP even, zero padded) matrix in LDS.  On
// return A holds the eigenvalues on its diagonal and V the eigenvectors.
template <int KMAX, int NT>
__device__ void jacobi_lds(double* A, double* V, int K, int KP, double* rc, double* rs, double* rt,
                           int* rp, int* rq, double* red) {
  const int tid = threadIdx.x;
  const int half = KP / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = tid; idx < K * K; idx += NT) {
      const int i = idx / K, j = idx - (idx / K) * K;
      const double a = A[i * KMAX + j];
      tot += a * a;
      if (i != j) off += a * a;
    }
    off = block_sum<NT>(off, red);
    tot = block_sum<NT>(tot, red);
    if (!(off > 1e-32 * tot)) break;   // off(A) <= 1e-16 ||A||_F (also stops on 0 or NaN)
    for (int r = 0; r < KP - 1; ++r) {
      if (tid < half) {
        int p, q;
        if (tid == 0) {
          p = 0;
          q = 1 + (r % (KP - 1));
        } else {
          p = 1 + ((tid + r) % (KP - 1));
          q = 1 + ((KP - 1 - tid + r) % (KP - 1));
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c, s, t;
        schur2(A[p * KMAX + p], A[q * KMAX + q], A[p * KMAX + q], c, s, t);
        rp[tid] = p;
        rq[tid] = q;
        rc[tid] = c;
        rs[tid] = s;
        rt[tid] = t;
      }
      __syncthreads();
      // A <- J^T A J on disjoint 2x2 blocks; V <- V J
      for (int idx = tid; idx < half * half; idx += NT) {
        const int a = idx / half, bq = idx - (idx / half) * half;
        const int pa = rp[a], qa = rq[a], pb = rp[bq], qb = rq[bq];
        if (a == bq) {
          const double t = rt[a];
          const double apq = A[pa * KMAX + qa];
          A[pa * KMAX + pa] -= t * apq;
          A[qa * KMAX + qa] += t * apq;
          A[pa * KMAX + qa] = 0.0;
          A[qa * KMAX + pa] = 0.0;
        } else {
          const double ca = rc[a], sa = rs[a], cb = rc[bq], sb = rs[bq];
          const double x00 = A[pa * KMAX + pb], x01 = A[pa * KMAX + qb];
          const double x10 = A[qa * KMAX + pb], x11 = A[qa * KMAX + qb];
          const double y00 = ca * x00 - sa * x10, y01 = ca * x01 - sa * x11;
          const double y10 = sa * x00 + ca * x10, y11 = sa * x01 + ca * x11;
          A[pa * KMAX + pb] = y00 * cb - y01 * sb;
          A[pa * KMAX + qb] = y00 * sb + y01 * cb;
          A[qa * KMAX + pb] = y10 * cb - y11 * sb;
          A[qa * KMAX + qb] = y10 * sb + y11 * cb;
        }
      }
      for (int idx = tid; idx < KP * half; idx += NT) {
        const int i = idx / half, bq = idx - (idx / half) * half;
        const int pb = rp[bq], qb = rq[bq];
        const double cb = rc[bq], sb = rs[bq];
        const double vp = V[i * KMAX + pb], vq = V[i * KMAX + qb];
        V[i * KMAX + pb] = cb * vp - sb * vq;
        V[i * KMAX + qb] = sb * vp + cb * vq;
      }
      __syncthreads();
    }
  }
}

// Select the cheaper side of the spectrum: Pi_+(Y) = sum_{l>0} lam_l v v^T
// = Y - sum_{l<0} lam_l v v^T.  Fills sel[0..nsel) and returns sign flag
// (1 = positive side).  Runs on thread 0 only; result broadcast via LDS.
template <int NT>
__device__ void choose_side(const double* A, int K, int KMAX_, int* sel, int* meta) {
  if (threadIdx.x == 0) {
    int npos = 0;
    for (int l = 0; l < K; ++l) npos += (A[l * KMAX_ + l] > 0.0);
    const int pos = (npos <= K - npos) ? 1 : 0;
    int n = 0;
    for (int l = 0; l < K; ++l) {
      const double lam = A[l * KMAX_ + l];
      if (pos ? (lam > 0.0) : (lam < 0.0)) sel[n++] = l;
    }
    meta[0] = n;
    meta[1] = pos;
  }
  __syncthreads();
}

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
