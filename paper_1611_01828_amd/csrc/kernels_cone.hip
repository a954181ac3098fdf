// Conic step (eq. Step2, PSD part) fused with the dual update (eq. Step3)
// for the cliques routed to it (up to kJacobiMax = 64 vertices; the shapes
// of a 96-vertex bucket are kept): one workgroup per clique, the block held
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
// Warm start (d.warm_v set): V starts from the clique's eigenvectors of the
// previous iteration and Y is rotated to V^T Y V before the sweeps; the
// rotations then accumulate onto that V, which is stored back for the next
// iteration.
// With relaxed steps 2-3 u_s and v+ are the blends of slot_arg / slot_vnew,
// H_k reads u_hat_x (xh) for them and x+ for the residual.
//
// T is the working precision of the eigen-decomposition (double, or float
// for the FP32 variant): Y is gathered and s+, z+, v+ are formed in double,
// and Pi_+(Y) = Y - sum_{lam<0} lam v v^T keeps Y exact when the negative
// side is the smaller one.  NT (threads per clique) is the tile shape the
// autotuner chooses per bucket.
#include "cone_common.h"

namespace cdcs {

template <int KMAX, int NT, typename T>
__global__ __launch_bounds__(NT) void k_cone_jacobi(DevPlan d, const int32_t* tasks) {
  __shared__ T A[KMAX * KMAX];
  __shared__ T V[KMAX * KMAX];
  __shared__ T G[sizeof(T) == 4 ? KMAX * KMAX : 1];   // FP32 warm start: V^T V
  __shared__ JacRot<KMAX, T> rot;
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
      yv = slot_arg(d, d.s[sl], d.z[sl], d.v[sl], d.xh[d.slot2ent[sl]]);
      if (a != bq) yv *= kInvSqrt2;
    }
    A[i * KMAX + j] = (T)yv;
    V[i * KMAX + j] = (i == j) ? T(1) : T(0);
  }
  __syncthreads();
  T* vstore = nullptr;
  if (d.warm_v) {
    vstore = static_cast<T*>(d.warm_v) + d.warm_off[k];
    const int32_t* sti = d.st + inst * kNst;
    if (sti[ST_WARM] && sti[ST_ITER] % kWarmRestart != 0) {
      for (int idx = tid; idx < K * K; idx += NT) {
        const int i = idx / K, j = idx - (idx / K) * K;
        V[i * KMAX + j] = vstore[idx];
      }
      __syncthreads();
      // FP32: the stored rotations lose orthogonality at float rounding per
      // iteration, cumulatively; one Newton-Schulz step restores it
      if constexpr (sizeof(T) == 4) orthonormalize_lds<KMAX, NT, T>(V, G, K);
      similarity_lds<KMAX, NT, T>(A, V, K);
    }
  }
  jacobi_lds<KMAX, NT, T>(A, V, K, KP, rot, red);
  choose_side<NT, T>(A, K, KMAX, sel, meta);
  const int nsel = meta[0], pos = meta[1];
  if (vstore)
    for (int idx = tid; idx < K * K; idx += NT) {
      const int i = idx / K, j = idx - (idx / K) * K;
      vstore[idx] = V[i * KMAX + j];
    }
  // epilogue over packed slots
  const int nslot = K * (K + 1) / 2;
  double ex = 0.0, ev = 0.0;
  for (int t = tid; t < nslot; t += NT) {
    int a, bq;
    unpack_index(t, K, a, bq);
    double acc = 0.0;
    for (int u = 0; u < nsel; ++u) {
      const int l = sel[u];
      acc += (double)V[a * KMAX + l] * (double)A[l * KMAX + l] * (double)V[bq * KMAX + l];
    }
    const int64_t sl = s0 + t;
    const double sv = d.s[sl], zv = d.z[sl], vv = d.v[sl];
    const int e = d.slot2ent[sl];
    const double xh = d.xh[e];
    const double xv = d.relax ? d.x[e] : xh;                 // (H x+) at the slot
    const double yvec = slot_arg(d, sv, zv, vv, xh);          // svec(Y) entry
    const double sc = (a == bq) ? 1.0 : kSqrt2;
    const double sp = pos ? acc * sc : yvec - acc * sc;      // svec(Pi_+(Y))
    const double zn = sp - yvec;
    const double vn = slot_vnew(d, sv, zv, vv, xh);
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
template <int KMAX, int NT, typename T>
__global__ __launch_bounds__(NT) void k_psd_jacobi(const int32_t* sizes, const int64_t* offs,
                                                   const int32_t* tasks, const double* in,
                                                   double* out) {
  __shared__ T A[KMAX * KMAX];
  __shared__ T V[KMAX * KMAX];
  __shared__ JacRot<KMAX, T> rot;
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
    A[i * KMAX + j] = (T)yv;
    V[i * KMAX + j] = (i == j) ? T(1) : T(0);
  }
  __syncthreads();
  jacobi_lds<KMAX, NT, T>(A, V, K, KP, rot, red);
  choose_side<NT, T>(A, K, KMAX, sel, meta);
  const int nsel = meta[0], pos = meta[1];
  const int nslot = K * (K + 1) / 2;
  for (int t = tid; t < nslot; t += NT) {
    int a, bq;
    unpack_index(t, K, a, bq);
    double acc = 0.0;
    for (int u = 0; u < nsel; ++u) {
      const int l = sel[u];
      acc += (double)V[a * KMAX + l] * (double)A[l * KMAX + l] * (double)V[bq * KMAX + l];
    }
    const double sc = (a == bq) ? 1.0 : kSqrt2;
    const double yvec = in[o + t];
    out[o + t] = pos ? acc * sc : yvec - acc * sc;   // each element read, then written, by one thread
  }
}

// tile shapes: (KMAX, threads per clique) candidates per bucket
namespace {
template <int KMAX, int NT, typename T>
void cone_launch(const DevPlan& d, const int32_t* tasks, int32_t ntask, hipStream_t st) {
  hipLaunchKernelGGL((k_cone_jacobi<KMAX, NT, T>), dim3(ntask), dim3(NT), 0, st, d, tasks);
}
template <int KMAX, int NT, typename T>
void psd_launch(const int32_t* sizes, const int64_t* offs, const int32_t* tasks, int32_t ntask, const double* in,
                double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_psd_jacobi<KMAX, NT, T>), dim3(ntask), dim3(NT), 0, st, sizes, offs, tasks, in, out);
}
// the bucket of KMAX; every thread count is a whole number of waves (the
// block reductions need it)
int bucket_kmax(int kmax) { return kmax <= 16 ? 16 : kmax <= 32 ? 32 : kmax <= 64 ? 64 : 96; }
}  // namespace

int jacobi_threads(int kmax, int variant) {
  switch (bucket_kmax(kmax)) {
    case 16: return variant ? 128 : 64;
    case 32: return variant ? 64 : 128;
    case 64: return variant ? 128 : 256;
    default: return variant ? 256 : 512;
  }
}

#define CDCS_CONE_DISPATCH(CALL, T)                       \
  switch (bucket_kmax(kmax) * 2 + (variant ? 1 : 0)) {    \
    case 32: CALL(16, 64, T); break;                      \
    case 33: CALL(16, 128, T); break;                     \
    case 64: CALL(32, 128, T); break;                     \
    case 65: CALL(32, 64, T); break;                      \
    case 128: CALL(64, 256, T); break;                    \
    case 129: CALL(64, 128, T); break;                    \
    case 192: CALL(96, 512, T); break;                    \
    default: CALL(96, 256, T); break;                     \
  }

void launch_cone_jacobi(const DevPlan& d, const int32_t* tasks, int32_t ntask, int kmax, int variant, int fp32,
                        hipStream_t st) {
  if (ntask <= 0) return;
#define CONE_CALL(KM, NTH, T) cone_launch<KM, NTH, T>(d, tasks, ntask, st)
  if (fp32) {
    CDCS_CONE_DISPATCH(CONE_CALL, float)
  } else {
    CDCS_CONE_DISPATCH(CONE_CALL, double)
  }
#undef CONE_CALL
}

void launch_psd_project(const int32_t* sizes, const int64_t* offs, const int32_t* tasks, int32_t ntask, int kmax,
                        const double* in, double* out, hipStream_t st, int variant, int fp32) {
  if (ntask <= 0) return;
#define PSD_CALL(KM, NTH, T) psd_launch<KM, NTH, T>(sizes, offs, tasks, ntask, in, out, st)
  if (fp32) {
    CDCS_CONE_DISPATCH(PSD_CALL, float)
  } else {
    CDCS_CONE_DISPATCH(PSD_CALL, double)
  }
#undef PSD_CALL
}

#undef CDCS_CONE_DISPATCH

}  // namespace cdcs
