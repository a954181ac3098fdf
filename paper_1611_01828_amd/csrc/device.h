// Device-side layout of a batched HSDE-ADMM solve on gfx950.
//
// All instances of a batch are concatenated: "entry space" (svec over the
// chordal pattern E'), "slot space" (the clique blocks s, z, v) and "row
// space" (constraints).  Kernels work on block descriptors that never
// straddle an instance, so every reduction has a fixed per-instance block
// range and a fixed summation order (bitwise reproducible, no atomics).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdcs {

constexpr int kThreads = 256;        // block size of the streaming kernels
constexpr int kEntChunk = 1024;      // entries per entry block
constexpr int kRowChunk = 64;        // constraint rows per row block (4 waves)
constexpr int kJacobiMax = 64;       // largest clique handled by the LDS Jacobi kernel (larger: tridiagonal path)

// per-instance scalar slots (double sc[B * kNsc])
enum Sc {
  SC_TAU = 0, SC_KAPPA, SC_DEN, SC_CTZX, SC_BTZY, SC_NB, SC_NC, SC_GAMMA, SC_OMEGA3, SC_BW,
  SC_CPX, SC_EPS_P, SC_EPS_D, SC_EPS_G, SC_CX, SC_BY, SC_PRI2, SC_DUA2, SC_PINF2, SC_DINF2,
  SC_UTAU, kNsc = 24
};

// status words per instance
// (ST_WARM: the cliques' stored eigenvectors belong to this instance's
// previous iteration; cleared at setup and by a restored state)
enum St { ST_STATUS = 0, ST_FROZEN, ST_ITER, ST_WARM, kNst = 4 };

constexpr int kWarmRestart = 64;     // warm-started Jacobi: a cold start every this many iterations

struct DevPlan {
  int32_t B;
  int32_t M;
  int64_t NE, NS;
  int32_t P;
  // per instance
  const int64_t* ent_off;     // B+1
  const int32_t* row_off;     // B+1
  const int32_t* clq_off;     // B+1
  const int32_t* eblk_off;    // B+1 (entry-block ranges)
  const int32_t* rblk_off;    // B+1 (row-block ranges)
  double* sc;                 // B * kNsc
  int32_t* st;                // B * kNst
  // entry space
  double* x;
  double* hsum;               // H^T (s + z + v) / 2
  double* q;                  // P^{-1} r0
  double* px;                 // P^{-1}(r0 - A^T w')
  double* atw;                // A^T w'
  const double* c;
  const double* pinv;         // 1 / (1 + D/2)
  const double* halfD;        // D / 2
  const double* zt_x;         // x part of M^{-1} zeta
  const double* atzy;         // A^T (y part of M^{-1} zeta)
  const int32_t* ent_sptr;    // NE+1: slots covering each entry (H^T as CSR)
  const int32_t* ent_slots;
  // over-relaxation of steps 2-3 (relax = alpha != 1); with relax the step-1
  // point u_hat_x is kept apart from x+ in xh, and the products of the
  // previous iterate A x, A^T y, H^T v are formed in the passes that already
  // read those operands.  Without relax xh aliases x and the others are null.
  double alpha;
  int32_t relax;
  double* xh;                 // u_hat_x
  double* atyo;               // A^T y (previous iterate)
  double* hvo;                // H^T v (previous iterate)
  double* axo;                // A x   (previous iterate), row space
  // warm-started Jacobi (null when off): each Jacobi clique's eigenvectors
  // of the previous iteration, K x K row-major in the working precision, at
  // warm_off[clique] elements into warm_v
  void* warm_v;
  const int64_t* warm_off;
  // slot space
  double* s;
  double* z;
  double* v;
  const int32_t* slot2ent;    // H as an index map
  // row space
  double* y;
  double* g;                  // right-hand side of the m x m solve
  double* w;                  // its solution w'
  const double* b;
  const double* zt_y;
  const int32_t* a_ptr;       // A, CSR over global entries
  const int32_t* a_col;
  const double* a_val;
  const int32_t* at_ptr;      // A^T, CSR over global rows
  const int32_t* at_row;
  const double* at_val;
  // A^T again, sliced ELL for k_spmv_at: the entries of every entry block,
  // sorted by their count of nonzeros (descending), are cut into chunks of
  // 64; chunk c stores its k-th nonzeros of the 64 lanes at
  // at_chptr[c] + 64 k + lane (zero-padded to the chunk's longest, its
  // first), so that a wave reads 64 consecutive values per step.
  const int32_t* at_choff;    // n_eblk: first chunk of each entry block
  const int64_t* at_chptr;    // chunks: offset into at_srow / at_sval
  const int32_t* at_chlen;    // chunks: nonzeros of the chunk's longest entry
  const int32_t* at_sent;     // chunks x 64: the lane's entry, or -1
  const int32_t* at_srow;
  const double* at_sval;
  // m x m factor per instance
  const int32_t* f_mode;      // 0 dense, 1 sparse, 2 dense with K^{-1} cached (small m)
  const int64_t* f_dense_off; // offset of the dense column-major factor
  const double* f_Ld;
  const double* f_Ldt;        // the transposes of the dense factors (same offsets)
  const double* f_Kinv;       // mode 2: K^{-1} = L^{-T} L^{-1}, m x m (same offsets)
  int32_t trsv_rows;          // rows per thread the dense sweeps need (1, 2, 4 or 8)
  const int32_t* f_perm;      // at row_off (local indices)
  const double* f_diag;       // at row_off
  const int32_t* f_lptr;      // at row_off + inst (m+1 each), values global into lcol
  const int32_t* f_lcol;
  const double* f_lval;
  const int32_t* f_uptr;
  const int32_t* f_ucol;
  const double* f_uval;
  const int32_t* f_flev_off;  // B+1 offsets into flev_ptr
  const int32_t* f_flev_ptr;  // values global into flev_rows
  const int32_t* f_flev_rows;
  const int32_t* f_blev_off;
  const int32_t* f_blev_ptr;
  const int32_t* f_blev_rows;
  double* trsv_z;             // M: the sparse solve's vector for orders above its LDS capacity
  // work lists
  const int4* eblk;           // {inst, begin, end, 0}
  int32_t n_eblk;
  const int4* rblk;
  int32_t n_rblk;
  // partial sums
  double* part_e;             // n_eblk * 4: [c.px, dres^2, (dres + tau c)^2, c.x]
  double* part_r;             // n_rblk * 4: [pres^2, (Ax)^2, b.y, 0]
  double* part_c;             // P * 2: [(Hx - s)^2, (v - z)^2]
  // cliques
  const int32_t* clq_size;
  const int64_t* clq_slot;    // first slot of each clique (global)
  const int32_t* clq_inst;
  // large-clique workspace
  double* big_work;
  const int64_t* big_off;     // per large task: offset into big_work
  const int32_t* big_size;    // per large task: clique order (tasks sorted by it, descending)
};

// doubles of workspace one large-clique task needs (matrix, eigenvectors,
// LU / panel scratch, tridiagonal data, tile partials)
// reflectors of the band-to-tridiagonal stage: kBandRefl doubles (tau and
// v_1..v_7) per step, (K + 6) / 8 steps per sweep, K - 2 sweeps
inline int64_t band_refl_size(int K) { return K > 2 ? (int64_t)(K - 2) * ((K + 6) / 8) * 8 : 0; }
inline int64_t large_work_size(int K) {
  const int64_t T = (K + 31) / 32;
  const int64_t ld = (K + 7) & ~7;
  return 5LL * ld * ld + 5LL * ld + 16 + T * (T + 1) + 64 + band_refl_size(K);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum in a fixed order (wave tree, then waves in order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  static_assert(NT >= 64 && NT % 64 == 0, "block_sum needs whole waves");
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += red[i];
    red[NT / 64] = t;
  }
  __syncthreads();
  return red[NT / 64];
}

// Steps 2-3 at one clique slot.  Step 1 in the eliminated form gives
// u_hat_s = (s + z - v + xh)/2 and u_hat_v = (s + z + v - xh)/2, with xh the
// slot's entry of H u_hat_x (h = r = w = 0).  Step 2 projects Y = ub_s - z and
// sets v+ = ub_v, where ub = u_hat (eqs. Step2-Step3) or, relaxed,
// ub = u + alpha (u_hat - u).  Without relaxation the paper's form is
// evaluated as such (Y = (s - z - v + xh)/2).
__device__ __forceinline__ double slot_arg(const DevPlan& d, double s, double z, double v, double xh) {
  if (!d.relax) return 0.5 * (s - z - v + xh);
  const double us = 0.5 * (s + z - v + xh);
  return (s + d.alpha * (us - s)) - z;
}
__device__ __forceinline__ double slot_vnew(const DevPlan& d, double s, double z, double v, double xh) {
  const double uv = 0.5 * (s + z + v - xh);
  return d.relax ? v + d.alpha * (uv - v) : uv;
}

// primal-only / dual-only ADMM (kernels_split.hip): arguments beyond the
// shared plan
struct SplitArgs {
  double rho;             // penalty of the consensus constraint
  double* w;              // slot space: projection argument
  double* p;              // slot space: projection result
  double* part_s;         // n_sblk * kSplitParts partial sums
  const int4* sblk;       // slot blocks {inst, begin, end, 0}
  int32_t n_sblk;
  const int32_t* sblk_off;  // B+1 (slot-block ranges)
};
constexpr int kSplitParts = 8;
constexpr int kSlotChunk = 4096;     // slots per slot block

// Restarted-GMRES bookkeeping of one instance per thread, on the device, so
// that a cycle runs without a host round trip.  Per instance i: the
// (R+1) x R Hessenberg matrix (column-major), the Givens rotations, the
// rotated right-hand side gamma, jlim (-1 while the instance still takes
// columns, else the number of columns its update uses), done, and a ring of
// the last kGmWindow restart residuals for the stall test.
struct GmState {
  double* H;      // B (R+1) R
  double* cs;     // B R
  double* sn;     // B R
  double* gam;    // B (R+1)
  double* hist;   // B kGmWindow
  double* gnorm;  // B
  int32_t* jlim;  // B
  int32_t* done;  // B
  int32_t* nhist; // B
  int32_t* alldone;  // 1
};
constexpr int kGmWindow = 5;
constexpr double kGmStall = 0.9;
void launch_gm_begin(const GmState& g, const double* nrm, double* scale, int B, int R, double tol, hipStream_t st);
void launch_gm_step(const GmState& g, const double* d1, const double* d2, const double* nrm, double* scale, int B,
                    int R, int j, double tol, hipStream_t st);
void launch_gm_solve(const GmState& g, double* coef, int B, int R, int jdone, hipStream_t st);
void launch_gm_final(const GmState& g, const double* nrm, double* resid, int32_t* reason, int B, double tol,
                     hipStream_t st);

// launchers (defined in the .hip files)
void launch_r0(const DevPlan& d, hipStream_t st);
void launch_spmv_a(const DevPlan& d, hipStream_t st);
void launch_trsv(const DevPlan& d, hipStream_t st);
void launch_spmv_at(const DevPlan& d, hipStream_t st);
void launch_scalar1(const DevPlan& d, hipStream_t st);
void launch_update_e(const DevPlan& d, hipStream_t st);
void launch_update_r(const DevPlan& d, hipStream_t st);
void launch_scalar2(const DevPlan& d, double eps_tol, int32_t max_iter, int32_t stop, hipStream_t st);
void launch_split_r(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st);
void launch_split_g(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st);
void launch_split_x(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st);
void launch_split_w(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st);
void launch_split_update(const DevPlan& d, const SplitArgs& a, int primal, hipStream_t st);
void launch_split_scalar(const DevPlan& d, const SplitArgs& a, double eps_tol, int32_t max_iter, int32_t stop,
                         hipStream_t st);
// cone step: tasks are clique ids.  Jacobi tile shape per bucket: variant 0
// = the default threads per clique, 1 = the other candidate (twice as many for
// 16-vertex cliques, half as many otherwise); fp32 = 1 runs the
// eigen-decomposition in FP32.
int jacobi_threads(int kmax, int variant);
void launch_cone_jacobi(const DevPlan& d, const int32_t* tasks, int32_t ntask, int kmax, int variant, int fp32,
                        hipStream_t st);
// large cliques: gather, tridiag, eig, backtrans, recon, partials
constexpr int kLargeSteps = 6;
// timing of the large-clique launches (kind 0 symv, 1 update, 2 trailing
// update, 3 tail in LDS, 4 eigen prep, 5 bisection, 6 isolated vectors,
// 7 clustered vectors, 8 WY factors, 9 back-transformation, 10 band panel
// QR, 11 band trailing update, 12 bulge chasing, 13 bulge-chasing
// back-transformation): begin() hands out an event
// pair that the launch itself records (the kernel's own start and end),
// end() files it
struct LaunchHook {
  void (*begin)(void* ctx, int kind, hipEvent_t* start, hipEvent_t* stop);
  void (*end)(void* ctx, int kind);
  void* ctx;
};
// Cliques of at least band_min vertices take the two-stage reduction (dense
// to band, band to tridiagonal); the others the one-stage blocked reduction
// and the LDS tail.
constexpr int kBandMinDefault = 137;
// host_sizes: the tasks' clique orders on the host, sorted descending
void launch_cone_large_step(const DevPlan& d, const int32_t* tasks, int32_t ntask, int32_t kmax,
                            const int32_t* host_sizes, int step, hipStream_t st, int band_min,
                            const LaunchHook* hook = nullptr);
// stand-alone projection of packed blocks
void launch_psd_project(const int32_t* sizes, const int64_t* offs, const int32_t* tasks, int32_t ntask,
                        int kmax, const double* in, double* out, hipStream_t st, int variant = 0, int fp32 = 0);
// tasks sorted by block order, descending; task_sizes (device) and
// host_sizes (host) hold those orders
void launch_psd_project_large(const int32_t* sizes, const int64_t* offs, const int32_t* tasks,
                              const int32_t* task_sizes, const int32_t* host_sizes, int32_t ntask, int32_t kmax,
                              const double* in, double* out, double* work, const int64_t* work_off, hipStream_t st,
                              int band_min = kBandMinDefault);

}  // namespace cdcs
