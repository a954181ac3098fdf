// Conic step (eq. Step2, PSD part) for cliques of 97..1024 vertices.
//
// Pi_+(Y) = sum_{lambda_l > 0} lambda_l v_l v_l^T = Y - sum_{lambda_l < 0} lambda_l v_l v_l^T,
// so only the eigenpairs of the smaller-signed side of the spectrum are
// computed.  Per clique (one task):
//   1. gather      Y (K x K, column-major) from the clique's slots
//   2. tridiag     Q^T Y Q = T by Householder reflections, blocked in panels
//                  of 32 columns with deferred rank-2k updates (the LAPACK
//                  sytrd/latrd scheme, Golub & Van Loan Section 8.3.1)
//   3. eig         Sturm-sequence bisection for the chosen eigenvalues
//                  (Golub & Van Loan Section 8.4.1), inverse iteration with
//                  a partially pivoted tridiagonal LU for the eigenvectors,
//                  re-orthogonalised within clusters of close eigenvalues
//                  (Peters & Wilkinson; Golub & Van Loan Section 8.2.2)
//   4. backtrans   V = Q Z, applying the stored reflectors
//   5. recon       the low-rank sum above on 32 x 32 output tiles, fused with
//                  s+, z+ = s+ - Y, v+ and the residual partial sums (ADMM
//                  mode) or written to the output blocks (projection mode)
//   6. partials    per-clique sum of the tile partials (fixed order)
#include <hip/hip_ext.h>

#include <algorithm>

#include "device.h"

namespace cdcs {

namespace {

constexpr int kLT = 1024;        // threads of the per-task kernels
constexpr int kTT = 512;         // threads of the tridiagonalisation kernel
constexpr int kNB = 32;          // panel width of the tridiagonalisation
constexpr int kBand = 8;         // bandwidth of the two-stage reduction's first stage
constexpr int kBandRefl = 8;     // doubles per stored bulge-chasing reflector: tau, v_1..v_7
// bulge-chasing steps per sweep (the first sweep's count; the stride of the
// reflector array)
__host__ __device__ __forceinline__ int band_nk(int K) { return (K + 6) / kBand; }
constexpr int kTile = 32;        // reconstruction tile
constexpr double kEps = 2.220446049250313e-16;
constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kInvSqrt2 = 0.70710678118654752;

__device__ __forceinline__ int packed_index(int a, int b, int K) {
  return b * K - (b * (b - 1)) / 2 + (a - b);
}

// workspace layout of one task (doubles), see large_work_size(); the
// matrix uses the padded leading dimension ld = K rounded up to 8
struct Ws {
  double* W;     // ld*ld matrix, then Householder vectors below the subdiagonal
  double* Z;     // ld*ld eigenvectors (first r columns, stride K)
  double* S;     // 3*ld*ld panel arrays / LU scratch
  double* d;     // ld    diagonal of T
  double* e;     // ld    off-diagonal of T
  double* tau;   // ld    reflector scalars
  double* lam;   // ld    chosen eigenvalues
  double* zs;    // ld    scale of each eigenvector column of Z (1 / its norm)
  double* meta;  // 16    [0] r, [1] 1 = positive side, [2] first, [3] pivmin, [4] ||T||
  double* tiles; // 2 * ntiles partial sums
  double* refl;  // band_refl_size(K): reflectors of the band-to-tridiagonal stage
};

__device__ __forceinline__ int lead_dim(int K) { return (K + 7) & ~7; }

__device__ __forceinline__ Ws ws_of(double* base, int K) {
  Ws w;
  const int ld = lead_dim(K);
  const size_t L2 = (size_t)ld * ld;
  w.W = base;
  w.Z = base + L2;
  w.S = base + 2 * L2;
  w.d = base + 5 * L2;
  w.e = w.d + ld;
  w.tau = w.e + ld;
  w.lam = w.tau + ld;
  w.zs = w.lam + ld;
  w.meta = w.zs + ld;
  w.tiles = w.meta + 16;
  const int T = (K + 31) / 32;
  w.refl = w.tiles + T * (T + 1) + 64;
  return w;
}

__device__ __forceinline__ double hash_unit(uint32_t a, uint32_t b) {
  uint64_t x = ((uint64_t)a << 32) ^ (uint64_t)b ^ 0x9E3779B97F4A7C15ull;
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;   // [-1, 1)
}

struct LargeArgs {
  // ADMM mode
  DevPlan d;
  const int32_t* tasks;       // clique ids (ADMM) or block ids (projection)
  // projection mode
  const int32_t* psizes;
  const int64_t* poffs;
  const double* pin;
  double* pout;
  // both
  double* work;
  const int64_t* woff;        // per task
  const int32_t* tsize;       // per task: order K of its block
  int band_min;               // tasks of at least this order take the two-stage reduction
};

template <bool ADMM>
__device__ __forceinline__ bool task_info(const LargeArgs& a, int task, int& K, int64_t& base) {
  const int k = a.tasks[task];
  if (ADMM) {
    if (a.d.st[a.d.clq_inst[k] * kNst + ST_FROZEN]) return false;
    K = a.d.clq_size[k];
    base = a.d.clq_slot[k];
  } else {
    K = a.psizes[k];
    base = a.poffs[k];
  }
  return true;
}

// svec(Y) entry of packed slot t of the task (ADMM: the argument of the
// projection of step 2, slot_arg)
template <bool ADMM>
__device__ __forceinline__ double yvec_of(const LargeArgs& a, int64_t base, int t) {
  if (ADMM) {
    const int64_t sl = base + t;
    return slot_arg(a.d, a.d.s[sl], a.d.z[sl], a.d.v[sl], a.d.xh[a.d.slot2ent[sl]]);
  }
  return a.pin[base + t];
}

}  // namespace

// ---------------------------------------------------------------------------
// 1. gather (full symmetric, padded rows zeroed): one workgroup per 32 x 32
//    tile of the lower triangle; the tile is read from the packed slots
//    column by column and written to both triangles through LDS, so that
//    every global access is coalesced
// ---------------------------------------------------------------------------
template <bool ADMM>
__global__ __launch_bounds__(256) void k_large_gather(LargeArgs a) {
  __shared__ double tile[kTile][kTile + 1];   // tile[col][row]
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  const int T = (K + kTile - 1) / kTile;
  const int q = blockIdx.y;
  if (q >= T * (T + 1) / 2) return;
  int tr = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while (tr * (tr + 1) / 2 > q) --tr;
  while ((tr + 1) * (tr + 2) / 2 <= q) ++tr;
  const int tc = q - tr * (tr + 1) / 2;
  const int i0 = tr * kTile, b0 = tc * kTile;   // rows i0.., columns b0.., i0 >= b0
  double* W = a.work + a.woff[blockIdx.x];
  const int ld = lead_dim(K);
  const int tid = threadIdx.x, il = tid & 31, g = tid >> 5;   // 8 column groups of 4
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int bl = g * 4 + u;
    const int i = i0 + il, b = b0 + bl;
    double y = 0.0;
    if (i < K && b < K && i >= b) {
      y = yvec_of<ADMM>(a, base, packed_index(i, b, K));
      if (i != b) y *= kInvSqrt2;
    }
    tile[bl][il] = y;
  }
  __syncthreads();
  const bool diag = tr == tc;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    // lower part: W(i, b) for column b, rows i (the mirror inside a diagonal tile)
    const int bl = g * 4 + u;
    const int i = i0 + il, b = b0 + bl;
    if (b < K && i < ld) W[(size_t)b * ld + i] = (diag && il < bl) ? tile[il][bl] : tile[bl][il];
  }
  if (!diag) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // upper part: W(b, i) = W(i, b) for column i, rows b
      const int rl = g * 4 + u;   // tile row -> column of the upper block
      const int i = i0 + rl, b = b0 + il;
      if (i < K) W[(size_t)i * ld + b] = tile[il][rl];
    }
  }
}

// ---------------------------------------------------------------------------
// 2. Householder tridiagonalisation (blocked panels of kNB columns, full
//    storage).  Column j of panel p (position i) is one pair of launches over
//    all tasks, so that each column step of a large clique is spread over
//    many workgroups (the step is a latency-bound matrix-vector product; one
//    workgroup per clique would leave most of the chip idle):
//      symv:   every workgroup forms the reflector of column j from the
//              column itself (H x = beta e_1, x = A(j+1:K, j)), then
//              y = A22 v on a chunk of 32 columns; the chunks past the
//              trailing columns give the panel dots t1 = Wp^T v, t2 = V^T v,
//              and each chunk leaves its share of y^T v
//      update: w = tau (y - V t1 - Wp t2) and Wp(:, i) = w + alpha v with
//              alpha = -tau/2 w^T v, where w^T v = tau (y^T v - 2 t1^T t2);
//              the Householder vector goes to column j, and column j + 1 is
//              brought up to date with the panel's reflectors 0..i
//      trail:  A22 -= V Wp^T + Wp V^T after the panel's last column
//    Kernel boundaries are the only synchronisation.  All global loads of
//    the symv are unconditional and aligned (double2 over the padded
//    leading dimension, zero padding rows, v zero outside its support).
// ---------------------------------------------------------------------------
constexpr int kSymvCols = 32;   // columns per symv workgroup (4 waves; 64 measured slower: 218 VGPRs)
constexpr int kWaveCols = kSymvCols / 4;
constexpr int kSymvRows = 256;  // rows per symv workgroup (2 steps of 128 per lane pair)
constexpr int kMaxRB = 1024 / kSymvRows;
constexpr int kUpdRows = 64;    // rows per update workgroup (4 waves split the panel sums)

constexpr int kMaxCB = (1024 + 2 * kNB + kSymvCols - 1) / kSymvCols;   // symv column chunks

struct TrdBufs {
  double* V;       // ld x kNB reflectors of the panel
  double* Wp;      // ld x kNB
  double* ypart;   // kMaxRB x ld   row-block partial sums of A22 v
  double* tpart;   // kMaxRB x 2 kNB partial panel dots t1, t2
  double* yvp;     // kMaxRB x kMaxCB  shares of y^T v per symv workgroup
  double* sspart;  // 1024 / kUpdRows  shares of ||x||^2 of the next column per update workgroup
  double* scl;     // 1      v = x / (alpha - beta) below row j + 1
};

__device__ __forceinline__ TrdBufs trd_bufs(const Ws& w, int ld) {
  TrdBufs b;
  b.V = w.S;
  b.Wp = w.S + (size_t)ld * kNB;
  b.ypart = w.S + (size_t)2 * ld * kNB;
  b.tpart = b.ypart + (size_t)kMaxRB * ld;
  b.yvp = b.tpart + kMaxRB * 2 * kNB;
  b.sspart = b.yvp + kMaxRB * kMaxCB;
  b.scl = b.sspart + 1024 / kUpdRows;
  return b;
}

// Once the trailing matrix has at most kTail columns it fits in LDS, and one
// workgroup per task finishes the reduction there (k_trd_tail).  The panel
// launches cover columns [0, trd_tail_start(K)), whole panels only.
constexpr int kTail = 136;   // full n x n storage of 136 columns: 148 KB of LDS
__host__ __device__ __forceinline__ int trd_tail_start(int K) {
  return (K > kTail) ? ((K - kTail + kNB - 1) / kNB) * kNB : 0;
}

// column j = p kNB + i of a task with K vertices, nb = columns of its panel
__device__ __forceinline__ bool trd_col(int K, int p, int i, int& j, int& nb) {
  const int j0 = p * kNB;
  if (j0 >= trd_tail_start(K)) return false;
  nb = min(kNB, K - 2 - j0);
  if (i >= nb) return false;
  j = j0 + i;
  return true;
}

// rows of the symv: from r0 = (j + 1) rounded down to even, in blocks of kSymvRows
__device__ __forceinline__ int trd_r0(int j) { return (j + 1) & ~1; }
__device__ __forceinline__ int trd_nrb(int j, int ld) { return (ld - trd_r0(j) + kSymvRows - 1) / kSymvRows; }

// The tridiagonalisation kernels only read and write the task's workspace,
// so they skip the frozen-instance test of task_info (a frozen instance's
// result is never reconstructed) and read the task's order from tsize: each
// of these launches is short, and every dependent global round trip before
// the first useful load shows in its duration.  For the same reason both
// kernels issue all their global loads before the first barrier.
template <bool ADMM>
__global__ __launch_bounds__(256, 4) void k_trd_symv(LargeArgs a, int p, int i, int ncy) {
  __shared__ __align__(16) double vbuf[1024];
  __shared__ double red[256 / 64 + 1];
  __shared__ double part[4];
  const int K = a.tsize[blockIdx.x];
  int j, nb;
  if (K >= a.band_min || !trd_col(K, p, i, j, nb)) return;
  const int ld = lead_dim(K);
  const int ncol = K - j - 1, nall = ncol + 2 * i;
  const int cb = blockIdx.y % ncy, rb = blockIdx.y / ncy;
  const int cbase = cb * kSymvCols;
  if (cbase >= nall || rb >= trd_nrb(j, ld)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const TrdBufs b = trd_bufs(w, ld);
  const double* W = w.W;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const bool lead = blockIdx.y == 0;
  // (1) this wave's operands: columns cbase + kWaveCols wid + u of
  //     [A22 | Wp(:, 0:i) | V(:, 0:i)] on rows rbase + [0, kSymvRows); W, V
  //     and Wp live in one workspace, every column addressed by its offset
  //     from W (V = W + 2 ld^2, Wp = V + kNB ld).  They do not depend on v.
  const int rbase = trd_r0(j) + rb * kSymvRows;
  const int cg = cbase + wid * kWaveCols;
  int coff[kWaveCols];
#pragma unroll
  for (int u = 0; u < kWaveCols; ++u) {
    const int q = min(cg + u, nall - 1);
    coff[u] = (q < ncol) ? (j + 1 + q) * ld
                         : 2 * ld * ld + ((q < ncol + i) ? (kNB + q - ncol) * ld : (q - ncol - i) * ld);
  }
  constexpr int NK = kSymvRows / 128;
  double2 av[NK][kWaveCols];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int rr = min(rbase + 2 * lane + 128 * k, ld - 2);
#pragma unroll
    for (int u = 0; u < kWaveCols; ++u) av[k][u] = *reinterpret_cast<const double2*>(W + coff[u] + rr);
  }
  // (2) column j: this workgroup's rows and columns of v, and ||x||^2 for
  //     x = A(j+1:K, j) (left in shares by the update of column j - 1, or
  //     summed here at the first column of a panel)
  const double alpha = W[(size_t)j * ld + j + 1];
  const double djj = W[(size_t)j * ld + j];
  constexpr int NR = kSymvRows / 256;   // rows of v each thread stages
  double xrow[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) xrow[q] = W[(size_t)j * ld + min(rbase + tid + 256 * q, K - 1)];
  double xcol[kWaveCols];
#pragma unroll
  for (int u = 0; u < kWaveCols; ++u) xcol[u] = W[(size_t)j * ld + min(j + 1 + cg + u, K - 1)];
  double ss = 0.0;
  if (i == 0) {
    for (int r = j + 2 + tid; r < K; r += 256) {
      const double x = W[(size_t)j * ld + r];
      ss += x * x;
    }
  }
  if (i == 0) {
    ss = block_sum<256>(ss, red);
  } else {
    // every wave sums the shares itself: one load per lane, no loop of
    // dependent loads
    const int nuc = (ld + kUpdRows - 1) / kUpdRows;
    const double t = b.sspart[min(lane, nuc - 1)];
    ss = wave_sum(lane < nuc ? t : 0.0);
  }
  // (3) reflector H = I - tau v v^T with H x = beta e_1 (every workgroup
  //     forms the same one)
  double beta, tu, scale;
  if (ss == 0.0) {
    beta = alpha;
    tu = 0.0;
    scale = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + ss), alpha);
    tu = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  auto vof = [&](int r, double x) { return (r == j + 1) ? 1.0 : ((r > j + 1 && r < K) ? x * scale : 0.0); };
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int rown = rbase + tid + 256 * q;
    if (rown < ld) vbuf[rown] = vof(rown, xrow[q]);
  }
  if (lead && tid == 0) {   // V(:, i) itself is written by the update launch
    w.d[j] = djj;
    w.e[j] = beta;
    w.tau[j] = tu;
    b.scl[0] = scale;
  }
  __syncthreads();
  double yv = 0.0;
  if (cg < nall) {
    // (4) y = A22 v and the panel dots on this block of rows
    double acc[kWaveCols];
#pragma unroll
    for (int u = 0; u < kWaveCols; ++u) acc[u] = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int r = rbase + 2 * lane + 128 * k;
      const int rr = min(r, ld - 2);
      const double2 vv = *reinterpret_cast<const double2*>(vbuf + rr);
      const double m = (r < ld) ? 1.0 : 0.0;
#pragma unroll
      for (int u = 0; u < kWaveCols; ++u) acc[u] += m * (av[k][u].x * vv.x + av[k][u].y * vv.y);
    }
#pragma unroll
    for (int u = 0; u < kWaveCols; ++u) {
      const double sum = wave_sum(acc[u]);
      const int q = cg + u;
      if (q < ncol) yv += sum * vof(j + 1 + q, xcol[u]);
      if (lane == 0 && q < nall) {
        if (q < ncol) b.ypart[(size_t)rb * ld + j + 1 + q] = sum;
        else if (q < ncol + i) b.tpart[rb * 2 * kNB + q - ncol] = sum;
        else b.tpart[rb * 2 * kNB + kNB + q - ncol - i] = sum;
      }
    }
  }
  if (lane == 0) part[wid] = yv;
  __syncthreads();
  if (tid == 0) b.yvp[rb * kMaxCB + cb] = (part[0] + part[1]) + (part[2] + part[3]);
}

template <bool ADMM>
__global__ __launch_bounds__(256) void k_trd_update(LargeArgs a, int p, int i) {
  __shared__ double t1[kNB], t2[kNB], cvj[kNB + 1], cwj[kNB + 1];
  __shared__ double red[256 / 64 + 1];
  __shared__ double py[4][kUpdRows], pv[4][kUpdRows];
  const int K = a.tsize[blockIdx.x];
  int j, nb;
  if (K >= a.band_min || !trd_col(K, p, i, j, nb)) return;
  const int ld = lead_dim(K);
  if (blockIdx.y * kUpdRows >= ld) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const TrdBufs b = trd_bufs(w, ld);
  const int tid = threadIdx.x;
  const bool next = i + 1 < nb;   // column j + 1 belongs to this panel
  const int jc = j + 1;
  const int nrb = trd_nrb(j, ld);
  const int nch = (K - j - 1 + 2 * i + kSymvCols - 1) / kSymvCols;
  // rows blockIdx.y * 64 + (tid & 63); the four waves split the panel sums
  const int rl = tid & 63, g = tid >> 6;
  const int r = blockIdx.y * kUpdRows + rl;
  const int rcl = min(r, ld - 1);
  const bool live = r > j && r < K;
  // global loads first
  constexpr int NM = kNB / 4;
  double Vr[NM], Wr[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int l = g + 4 * m;
    if (l < i) {
      Vr[m] = b.V[(size_t)l * ld + rcl];
      Wr[m] = b.Wp[(size_t)l * ld + rcl];
    } else {
      Vr[m] = 0.0;
      Wr[m] = 0.0;
    }
  }
  // fixed-count loops with clamped indices: the loads issue together
  double yrow = 0.0, yjc = 0.0;
#pragma unroll
  for (int q = 0; q < kMaxRB; ++q) {
    const size_t o = (size_t)min(q, nrb - 1) * ld;
    const double a0 = b.ypart[o + rcl], a1 = b.ypart[o + jc];
    yrow += (q < nrb) ? a0 : 0.0;
    yjc += (q < nrb) ? a1 : 0.0;
  }
  const double wjr = w.W[(size_t)jc * ld + rcl];
  const double xjr = w.W[(size_t)j * ld + rcl];
  const double scale = b.scl[0];
  double yv = 0.0;
  if (tid < nrb * nch) yv = b.yvp[(tid / nch) * kMaxCB + tid % nch];
  if (tid < i) {
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxRB; ++q) {
      const int o = min(q, nrb - 1) * 2 * kNB + tid;
      const double a1 = b.tpart[o], a2 = b.tpart[o + kNB];
      s1 += (q < nrb) ? a1 : 0.0;
      s2 += (q < nrb) ? a2 : 0.0;
    }
    t1[tid] = s1;
    t2[tid] = s2;
  }
  if (tid < i) {
    cvj[tid] = b.V[(size_t)tid * ld + jc];
    cwj[tid] = b.Wp[(size_t)tid * ld + jc];
  }
  if (tid == i) cvj[i] = 1.0;   // v(j + 1) = 1
  // y^T v (every workgroup forms the same sum); the barriers of the block
  // sum also publish t1, t2, cvj, cwj
  yv = block_sum<256>(yv, red);
  double tt = 0.0;
  for (int l = 0; l < i; ++l) tt += t1[l] * t2[l];
  const double tu = w.tau[j];
  const double al = -0.5 * tu * (tu * (yv - 2.0 * tt));
  // Wp(jc, i) as every workgroup forms it
  double wpj;
  {
    double y = yjc;
    for (int l = 0; l < i; ++l) y -= cvj[l] * t1[l] + cwj[l] * t2[l];
    wpj = tu * y + al * cvj[i];
  }
  double sy = 0.0, sv = 0.0;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int l = g + 4 * m;
    if (l < i) {
      sy += Vr[m] * t1[l] + Wr[m] * t2[l];
      sv += Vr[m] * cwj[l] + Wr[m] * cvj[l];
    }
  }
  py[g][rl] = sy;
  pv[g][rl] = sv;
  __syncthreads();
  double xx = 0.0;   // share of ||A(jc+2:K, jc)||^2 for the next reflector
  if (g == 0 && r < ld) {
    // v of column j on this row: V(:, i) and the Householder vector below
    // the subdiagonal
    const double vir = (r == j + 1) ? 1.0 : ((r > j + 1 && r < K) ? xjr * scale : 0.0);
    b.V[(size_t)i * ld + r] = vir;
    double wr = 0.0;
    if (live) {
      const double y = yrow - ((py[0][rl] + py[1][rl]) + (py[2][rl] + py[3][rl]));
      wr = tu * y + al * vir;
      if (next && r >= jc) {
        double v = wjr - ((pv[0][rl] + pv[1][rl]) + (pv[2][rl] + pv[3][rl]));
        v -= vir * wpj + wr * cvj[i];
        w.W[(size_t)jc * ld + r] = v;
        if (r >= jc + 2) xx = v * v;
      }
      if (r >= j + 2) w.W[(size_t)j * ld + r] = vir;   // Householder vector below the subdiagonal
    }
    b.Wp[(size_t)i * ld + r] = wr;
  }
  if (next) {
    xx = wave_sum(xx);   // wave 0 holds the workgroup's 64 rows
    if (tid == 0) b.sspart[blockIdx.y] = xx;
  }
}

template <bool ADMM>
__global__ __launch_bounds__(kTT) void k_trd_trail(LargeArgs a, int p) {
  __shared__ double stage[2 * kNB * 128 + 2 * kNB * 64];
  double(*pr_v)[128] = reinterpret_cast<double(*)[128]>(stage);
  double(*pr_w)[128] = reinterpret_cast<double(*)[128]>(stage + kNB * 128);
  double(*pc_v)[64] = reinterpret_cast<double(*)[64]>(stage + 2 * kNB * 128);
  double(*pc_w)[64] = reinterpret_cast<double(*)[64]>(stage + 2 * kNB * 128 + kNB * 64);
  const int K = a.tsize[blockIdx.x];
  const int j0 = p * kNB;
  if (K >= a.band_min || j0 >= trd_tail_start(K)) return;
  const int nb = kNB;
  const int jn = j0 + nb, n2 = K - jn;
  const int ntr = (n2 + 127) / 128, ntc = (n2 + 63) / 64;
  const int tile = blockIdx.y;
  if (tile >= ntr * ntc) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int ld = lead_dim(K);
  const TrdBufs b = trd_bufs(w, ld);
  double* W = w.W;
  const int tid = threadIdx.x;
  // A22 -= V Wp^T + Wp V^T on a 128 x 64 tile (both triangles), panel rows
  // staged in LDS, 4 x 4 outputs per thread
  // (staging and the final read-modify-write use clamped indices: loads
  // that sit behind a bounds test compile into one round trip each)
  const int r0 = jn + (tile % ntr) * 128, c0 = jn + (tile / ntr) * 64;
#pragma unroll
  for (int k = 0; k < 128 * kNB / kTT; ++k) {
    const int idx = tid + k * kTT, rr = idx & 127, l = idx >> 7;
    const size_t o = (size_t)l * ld + min(r0 + rr, K - 1);
    const double vv = b.V[o], ww = b.Wp[o];
    const bool ok = r0 + rr < K;
    pr_v[l][rr] = ok ? vv : 0.0;
    pr_w[l][rr] = ok ? ww : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 64 * kNB / kTT; ++k) {
    const int idx = tid + k * kTT, cc = idx & 63, l = idx >> 6;
    const size_t o = (size_t)l * ld + min(c0 + cc, K - 1);
    const double vv = b.V[o], ww = b.Wp[o];
    const bool ok = c0 + cc < K;
    pc_v[l][cc] = ok ? vv : 0.0;
    pc_w[l][cc] = ok ? ww : 0.0;
  }
  __syncthreads();
  const int tr = tid & 31, tc = tid >> 5;     // rows tr + 32 u, columns 4 tc + q
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[u][q] = 0.0;
  for (int l = 0; l < nb; ++l) {
    double cv[4], cw[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cv[q] = pc_v[l][4 * tc + q];
      cw[q] = pc_w[l][4 * tc + q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double rv = pr_v[l][tr + 32 * u], rw = pr_w[l][tr + 32 * u];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[u][q] += rv * cw[q] + rw * cv[q];
    }
  }
  double old[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      old[u][q] = W[(size_t)min(c0 + 4 * tc + q, K - 1) * ld + min(r0 + tr + 32 * u, K - 1)];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = r0 + tr + 32 * u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = c0 + 4 * tc + q;
      if (r < K && c < K) W[(size_t)c * ld + r] = old[u][q] - acc[u][q];
    }
  }
}

// The last columns [j0, K) of a task in LDS (full n x n storage, n <= TAIL),
// reduced column by column: x = A(c+1:n, c) gives the reflector, then
// p = tau A22 v, w = p - tau/2 (p^T v) v and A22 -= v w^T + w v^T
// (Golub & Van Loan Algorithm 8.3.1).  Thread (r, h) owns row r and the
// columns q = h mod TG (TG = TT / TR groups of TR row slots; the last
// threads of the block idle).  Two shapes: tails up to 136 columns (148 KB
// of LDS, 1024 threads, one workgroup per CU) and, for launches whose
// one-stage cliques have at most 64 vertices, tails up to 64 (35 KB, 256
// threads, four workgroups per CU).
template <bool ADMM, int TAIL, int TT, int TR>
__global__ __launch_bounds__(TT) void k_trd_tail(LargeArgs a) {
  constexpr int TG = TT / TR;
  static_assert(TR >= TAIL && TAIL <= 192 && TR * TG <= TT, "tail layout");
  __shared__ double A[TAIL * TAIL];
  __shared__ double vb[TAIL], wb[TAIL], ph[TG][TAIL];
  __shared__ double red[4];
  const int K = a.tsize[blockIdx.x];
  if (K >= a.band_min) return;   // tridiagonal after the two-stage reduction
  const int j0 = trd_tail_start(K), n = K - j0;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int ld = lead_dim(K);
  double* W = w.W;
  const int tid = threadIdx.x;
  const int r = tid % TR, h = tid / TR;   // h == TG: idle
  {
    // all of the thread's loads in flight together, from clamped in-range
    // addresses (entry min(idx, n^2 - 1) of the n x n block)
    constexpr int NL = (TAIL * TAIL + TT - 1) / TT;
    double x[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int idx = min(tid + TT * q, n * n - 1), c = idx / n, rr = idx - c * n;
      x[q] = W[(size_t)(j0 + c) * ld + j0 + rr];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) asm volatile("" : "+v"(x[q]));
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int idx = tid + TT * q;
      if (idx < n * n) A[idx] = x[q];
    }
  }
  __syncthreads();
  const int lane = tid & 63;
  for (int c = 0; c < n - 2; ++c) {
    const int j = j0 + c;
    // (1) wave 0: reflector of column c (rows lane + 64 u)
    if (tid < 64) {
      double xs[3], ss = 0.0;
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int rr = lane + 64 * u;
        xs[u] = (rr < n) ? A[c * n + rr] : 0.0;
        if (rr >= c + 2 && rr < n) ss += xs[u] * xs[u];
      }
      ss = wave_sum(ss);
      const double alpha = A[c * n + c + 1];
      double beta, tu, scale;
      if (ss == 0.0) {
        beta = alpha;
        tu = 0.0;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + ss), alpha);
        tu = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int rr = lane + 64 * u;
        const double vr = (rr == c + 1) ? 1.0 : ((rr > c + 1 && rr < n) ? xs[u] * scale : 0.0);
        if (rr < TAIL) vb[rr] = vr;
        if (rr >= c + 2 && rr < n) W[(size_t)j * ld + j0 + rr] = vr;   // Householder vector
      }
      if (lane == 0) {
        red[0] = tu;
        w.d[j] = A[c * n + c];
        w.e[j] = beta;
        w.tau[j] = tu;
      }
    }
    __syncthreads();
    const double tu = red[0];
    // (2) p = tau A22 v on rows and columns > c, column groups in ph
    const bool live = h < TG && r > c && r < n;
    double acc = 0.0;
    if (live)
      for (int q = c + 1 + h; q < n; q += TG) acc += A[q * n + r] * vb[q];
    if (h < TG && r < TAIL) ph[h][r] = acc;
    __syncthreads();
    // (3) wave 0: w = p - tau/2 (p^T v) v
    if (tid < 64) {
      double pr[3], pv = 0.0;
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int rr = lane + 64 * u;
        double t = 0.0;
        if (rr > c && rr < n) {
#pragma unroll
          for (int g = 0; g < TG; ++g) t += ph[g][rr];
          t *= tu;
          pv += t * vb[rr];
        }
        pr[u] = t;
      }
      pv = wave_sum(pv);
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int rr = lane + 64 * u;
        if (rr < TAIL) wb[rr] = (rr > c && rr < n) ? pr[u] - 0.5 * tu * pv * vb[rr] : 0.0;
      }
    }
    __syncthreads();
    // (4) A22 -= v w^T + w v^T
    if (live) {
      const double vr = vb[r], wr = wb[r];
      for (int q = c + 1 + h; q < n; q += TG) A[q * n + r] -= vr * wb[q] + wr * vb[q];
    }
    __syncthreads();
  }
  if (tid == 0) {
    w.d[K - 2] = A[(n - 2) * n + n - 2];
    w.d[K - 1] = A[(n - 1) * n + n - 1];
    w.e[K - 2] = A[(n - 2) * n + n - 1];
    w.e[K - 1] = 0.0;
    w.tau[K - 2] = 0.0;
    w.tau[K - 1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// 2'. Two-stage tridiagonalisation for cliques of at least band_min vertices
//    (successive band reduction: Bischof, Lang & Sun; the bulge chasing of
//    Schwarz's and Lang's band-to-tridiagonal algorithms):
//    stage 1 reduces Y to a band of width kBand.  Panel p (columns
//    j0 = 8p .. j0 + 7) takes the Householder QR of A(j0+8:K, j0:j0+8), then
//    the two-sided update A22 <- Q^T A22 Q of the trailing matrix with
//    Q = I - V T V^T: X = A22 V T, Y = X - 1/2 V T^T V^T X, A22 -= V Y^T +
//    Y V^T.  Column c keeps the band on rows c..c+8 and its reflector below
//    (1 on row c + 8, implicit), tau[c].  Stage 2 reduces the band to
//    tridiagonal form in LDS: sweep s annihilates column s below the
//    subdiagonal with a reflector on rows s+1..s+8, which fills a block
//    kBand rows further down; each further step annihilates the first column
//    of that bulge with a reflector on its rows and moves the fill another
//    kBand rows down.  The trailing matrix is read once per panel of kBand
//    columns (the one-stage reduction reads it once per column).
//    Launches per panel: k_band_panel (one workgroup per task: Y of the
//    previous panel, the panel's columns brought up to date, its QR, T and
//    U = V T) and k_band_trail (many workgroups: the previous panel's
//    trailing update fused with A22 U of this panel); then k_band_chase.
// ---------------------------------------------------------------------------
constexpr int kBandT = 256;                 // threads of the panel kernel (one wave per SIMD)
constexpr int kBandRows = 1024 / kBandT;    // rows per thread of the panel kernel
constexpr int kBandTile = 128;              // columns of a trailing-update tile (and of an A22 U partial)
constexpr int kChaseWaves = 8;              // waves of the bulge chasing (8 sweeps each; two per SIMD, so that a
                                            // new group of sweeps need not wait for a wave to finish its last)
constexpr int kChaseLd = 1032;              // LDS stride of a stored diagonal: K + 7 columns, zero past K
constexpr int kChaseSpin = 1 << 22;         // bound on a wave's wait for the previous sweep

// panels of a task: panel p is reduced while its QR block has two rows or more
__host__ __device__ __forceinline__ int band_panels(int K) { return (K - 9 + kBand - 1) / kBand; }

// (pointers computed from the parity rather than picked from an array, which
// would put the structure in scratch memory)
struct BandBufs {
  double* S;
  int ld;
  // ld x kBand, row-major: explicit reflectors of the panels of parity par
  __device__ double* V(int par) const { return S + (size_t)par * kBand * ld; }
  __device__ double* U() const { return S + (size_t)2 * kBand * ld; }   // V T of the current panel
  __device__ double* Y() const { return S + (size_t)3 * kBand * ld; }   // Y of the previous panel
  // kBand x kBand (row-major) per parity
  __device__ double* T(int par) const { return S + (size_t)4 * kBand * ld + par * kBand * kBand; }
  // per column tile, ld x kBand: partial sums of A22 U of the current panel
  __device__ double* X() const { return S + (size_t)4 * kBand * ld + 2 * kBand * kBand; }
};

__device__ __forceinline__ BandBufs band_bufs(const Ws& w, int ld) { return BandBufs{w.S, ld}; }

// per-lane values m[0..31] summed over the wave by recursive halving (32
// exchanges): lane L returns the total of value L & 31
template <int H>
__device__ __forceinline__ void halve_step(double (&m)[32], int lane) {
  const bool up = (lane & H) != 0;
#pragma unroll
  for (int q = 0; q < H; ++q) {
    const double send = up ? m[q] : m[q + H];
    const double keep = up ? m[q + H] : m[q];
    m[q] = keep + __shfl_xor(send, H, 64);
  }
}
__device__ __forceinline__ double wave_reduce_scatter32(double (&m)[32], int lane) {
  halve_step<16>(m, lane);
  halve_step<8>(m, lane);
  halve_step<4>(m, lane);
  halve_step<2>(m, lane);
  halve_step<1>(m, lane);
  return m[0] + __shfl_xor(m[0], 32, 64);
}

// (A^T B)(i, j) = sum over the block's rows of A(r, i) B(r, j) for the
// kBandRows x kBand row slices A, B of every thread, into out[64] (LDS,
// row-major); big: LDS scratch of kBandT doubles
__device__ __forceinline__ void band_gram(const double (&A)[kBandRows][kBand], const double (&B)[kBandRows][kBand],
                                          double (*big)[64], double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    double m[32];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jx = 0; jx < kBand; ++jx) {
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < kBandRows; ++u) t += A[u][4 * hf + i] * B[u][jx];
        m[i * kBand + jx] = t;
      }
    const double v = wave_reduce_scatter32(m, lane);
    if (lane < 32) big[wid][32 * hf + lane] = v;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kBandT / 64; ++q) t += big[q][threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// x of another lane through a DPP exchange (CTRL: the DPP control word; the
// controls used here read a valid lane for every lane, so the destination
// needs no initial value)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int l2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  const int h2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(h2, l2);
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}
// sum over the wave: DPP exchanges inside each row of 16 lanes (xor 1,
// xor 2, half-row mirror, row mirror), then the four row sums read from
// lanes 0, 16, 32 and 48 (every lane gets the total)
__device__ __forceinline__ double wave_sum_dpp(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x141>(x);
  x += dpp_f64<0x140>(x);
  return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

// block sums of NV values over kBandT threads (buf: one of two alternating
// buffers, so that consecutive sums need one barrier each)
// (values below k0 are left as they are; k0 is a constant after unrolling)
template <int NV>
__device__ __forceinline__ void band_block_sum(double (&v)[NV], double (*buf)[kBand], int k0 = 0) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if (k >= k0) v[k] = wave_sum_dpp(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k >= k0) buf[wid][k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < k0) continue;
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kBandT / 64; ++q) t += buf[q][k];
    v[k] = t;
  }
}

template <bool ADMM>
__global__ __launch_bounds__(kBandT) void k_band_panel(LargeArgs a, int p) {
  static_assert(kBand == 8 && kBandT * kBandRows == 1024 && kBandT > 8 + kBand, "panel layout");
  __shared__ double red[2][kBandT / 64][kBand];
  __shared__ double big[kBandT / 64][64];
  __shared__ double sm[64], st[64], cv[kBand][kBand], cy[kBand][kBand];
  __shared__ double piv[2][kBand], taus[kBand], tprev[kBand * kBand];
  const int K = a.tsize[blockIdx.x];
  if (K < a.band_min) return;
  const int np = band_panels(K);
  if (p > np) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int ld = lead_dim(K);
  const BandBufs bb = band_bufs(w, ld);
  double* W = w.W;
  const int tid = threadIdx.x;
  const int j0 = p * kBand, r0 = j0 + kBand;
  const int nc = min(kBand, K - j0);
  int nred = 0;
  // the panel's columns on rows j0 + tid + kBandT u, in registers (clamped
  // loads); loaded after the work on panel p - 1's Y, which does not need them
  double P[kBandRows][kBand];
  auto load_panel = [&]() {
#pragma unroll
    for (int u = 0; u < kBandRows; ++u)
#pragma unroll
      for (int l = 0; l < kBand; ++l)
        P[u][l] = W[(size_t)(j0 + min(l, nc - 1)) * ld + min(j0 + tid + kBandT * u, K - 1)];
  };
  if (p == 0) load_panel();
  if (p > 0) {
    // (a) Y of panel p - 1 on rows [j0, K): X = A22 U (the column-tile
    //     partials of k_band_trail summed), M = V^T X, Y = X - 1/2 V (T^T M)
    const double* Vq = bb.V((p + 1) & 1);
    // T of panel p - 1, its load issued with the others
    const double tq = (tid < 64) ? bb.T((p + 1) & 1)[tid] : 0.0;
    // (the partials of two column tiles loaded at a time for all of the
    // thread's rows, each batch issued together)
    const int nct = (K - j0 + kBandTile - 1) / kBandTile;
    double X[kBandRows][kBand], Vr[kBandRows][kBand];
#pragma unroll
    for (int u = 0; u < kBandRows; ++u) {
      const int r = j0 + tid + kBandT * u;
      const int rc = min(r, K - 1);
#pragma unroll
      for (int l = 0; l < kBand; ++l) {
        Vr[u][l] = (r < K) ? Vq[(size_t)rc * kBand + l] : 0.0;
        X[u][l] = 0.0;
      }
    }
    for (int h = 0; h < nct; h += 2) {
      double xp[kBandRows][2][kBand];
#pragma unroll
      for (int u = 0; u < kBandRows; ++u) {
        const int rc = min(j0 + tid + kBandT * u, K - 1);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int l = 0; l < kBand; ++l) xp[u][ct][l] = bb.X()[((size_t)min(h + ct, nct - 1) * ld + rc) * kBand + l];
      }
#pragma unroll
      for (int u = 0; u < kBandRows; ++u) {
        const bool ok = j0 + tid + kBandT * u < K;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int l = 0; l < kBand; ++l) X[u][l] += (ok && h + ct < nct) ? xp[u][ct][l] : 0.0;
      }
    }
    if (tid < 64) tprev[tid] = tq;
    band_gram(Vr, X, big, sm);   // M = V^T X (its barrier also publishes tprev)
    __syncthreads();
    if (tid < 64) {
      const int i = tid >> 3, jx = tid & 7;   // (T^T M)(i, jx)
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < kBand; ++k) t += tprev[k * kBand + i] * sm[k * kBand + jx];
      st[tid] = t;
    }
    __syncthreads();
    // (the empty asm statements keep the compiler from loading all of an
    // 8 x 8 LDS matrix into registers at once)
#pragma unroll
    for (int l = 0; l < kBand; ++l) {
      double sl[kBand];
#pragma unroll
      for (int i = 0; i < kBand; ++i) sl[i] = st[i * kBand + l];
#pragma unroll
      for (int u = 0; u < kBandRows; ++u) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < kBand; ++i) t += Vr[u][i] * sl[i];
        X[u][l] -= 0.5 * t;   // now Y
      }
      asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int u = 0; u < kBandRows; ++u) {
      const int r = j0 + tid + kBandT * u;
      if (r < K)
#pragma unroll
        for (int l = 0; l < kBand; ++l) bb.Y()[(size_t)r * kBand + l] = X[u][l];
    }
    // (b) the panel's columns (rows [j0, K)) brought up to date with panel
    //     p - 1: A(:, c) -= V Y(c, :)^T + Y V(c, :)^T
    load_panel();
    if (tid < kBand)
#pragma unroll
      for (int l = 0; l < kBand; ++l) {
        cv[tid][l] = Vr[0][l];
        cy[tid][l] = X[0][l];
      }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kBand; ++c) {
      double yc[kBand], vc[kBand];
#pragma unroll
      for (int l = 0; l < kBand; ++l) {
        yc[l] = cy[c][l];
        vc[l] = cv[c][l];
      }
#pragma unroll
      for (int u = 0; u < kBandRows; ++u) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < kBand; ++l) t += Vr[u][l] * yc[l] + X[u][l] * vc[l];
        P[u][c] -= t;
      }
      asm volatile("" ::: "memory");
    }
  }
  if (p == np) {
    // the last columns (at most 9 rows): band entries, no reflector
#pragma unroll
    for (int u = 0; u < kBandRows; ++u) {
      const int r = j0 + tid + kBandT * u;
      if (r < K)
#pragma unroll
        for (int l = 0; l < kBand; ++l)
          if (l < nc) W[(size_t)(j0 + l) * ld + r] = P[u][l];
    }
    if (tid < K - j0) w.tau[j0 + tid] = 0.0;
    return;
  }
  // (c) Householder QR of rows [r0, K) of the panel (rows [j0, r0) are its
  //     diagonal block, kept as they are); P(r, l) below the pivot then
  //     holds the Householder vector, R above.  One block sum per column:
  //     ss = sum_{t > rl} P(t, l)^2 and g_m = sum_{t > rl} P(t, l) P(t, m)
  //     (m > l), the pivot row broadcast beside it; v = (1, P(t, l) scale)
  //     then gives v^T P(:, m) = P(rl, m) + scale g_m.
#pragma unroll
  for (int l = 0; l < kBand; ++l) {
    const int rl = r0 + l;   // pivot row: thread kBand + l, u = 0
    if (rl >= K) {
      if (tid == 0) taus[l] = 0.0;
      continue;
    }
    double sg[kBand];
#pragma unroll
    for (int mm = 0; mm < kBand; ++mm) sg[mm] = 0.0;
#pragma unroll
    for (int u = 0; u < kBandRows; ++u) {
      const int r = j0 + tid + kBandT * u;
      const double x = (r > rl && r < K) ? P[u][l] : 0.0;
#pragma unroll
      for (int mm = l; mm < kBand; ++mm) sg[mm] += x * P[u][mm];
    }
    double* pv = piv[l & 1];
    if (tid == kBand + l)
#pragma unroll
      for (int mm = 0; mm < kBand; ++mm) pv[mm] = P[0][mm];
    band_block_sum<kBand>(sg, red[nred++ & 1], l);   // sums of columns l.. only
    const double alpha = pv[l];
    double beta, tu, scale;
    if (sg[l] == 0.0) {
      beta = alpha;
      tu = 0.0;
      scale = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sg[l]), alpha);
      tu = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    double wv[kBand];
#pragma unroll
    for (int mm = l + 1; mm < kBand; ++mm) wv[mm] = pv[mm] + scale * sg[mm];
#pragma unroll
    for (int u = 0; u < kBandRows; ++u) {
      const int r = j0 + tid + kBandT * u;
      const double vl = (r == rl) ? 1.0 : ((r > rl && r < K) ? P[u][l] * scale : 0.0);
#pragma unroll
      for (int mm = l + 1; mm < kBand; ++mm) P[u][mm] -= tu * vl * wv[mm];
      P[u][l] = (r == rl) ? beta : ((r > rl) ? vl : P[u][l]);
    }
    if (tid == 0) taus[l] = tu;
  }
  // (d) write back the diagonal block, R and the Householder vectors; the
  //     explicit V (1 on the pivot, zero above); tau
  double V[kBandRows][kBand];
#pragma unroll
  for (int u = 0; u < kBandRows; ++u) {
    const int r = j0 + tid + kBandT * u;
#pragma unroll
    for (int l = 0; l < kBand; ++l) {
      V[u][l] = (r == r0 + l) ? 1.0 : ((r > r0 + l && r < K) ? P[u][l] : 0.0);
      if (r < K) W[(size_t)(j0 + l) * ld + r] = P[u][l];
    }
    if (r >= r0 && r < K)
#pragma unroll
      for (int l = 0; l < kBand; ++l) bb.V(p & 1)[(size_t)r * kBand + l] = V[u][l];
  }
  // (e) T (forward, columnwise: T(k, i) = -tau_i sum_{k <= m < i} T(k, m)
  //     (V^T V)(m, i)) and U = V T
  __syncthreads();   // taus
  band_gram(V, V, big, sm);   // V^T V
  if (tid < kBand) w.tau[j0 + tid] = taus[tid];
  __syncthreads();
  if (tid < kBand) {
    const int k = tid;
    double tr[kBand];
#pragma unroll
    for (int i = 0; i < kBand; ++i) {
      double t = 0.0;
#pragma unroll
      for (int mm = 0; mm < kBand; ++mm)
        if (mm >= k && mm < i) t += tr[mm] * sm[mm * kBand + i];
      tr[i] = (i < k) ? 0.0 : ((i == k) ? taus[i] : -taus[i] * t);
    }
#pragma unroll
    for (int i = 0; i < kBand; ++i) {
      st[k * kBand + i] = tr[i];
      bb.T(p & 1)[k * kBand + i] = tr[i];
    }
  }
  __syncthreads();
  double Ur[kBandRows][kBand];
#pragma unroll
  for (int l = 0; l < kBand; ++l) {
    double sl[kBand];
#pragma unroll
    for (int k = 0; k < kBand; ++k) sl[k] = st[k * kBand + l];
#pragma unroll
    for (int u = 0; u < kBandRows; ++u) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < kBand; ++k) t += V[u][k] * sl[k];
      Ur[u][l] = t;
    }
    asm volatile("" ::: "memory");
  }
#pragma unroll
  for (int u = 0; u < kBandRows; ++u) {
    const int r = j0 + tid + kBandT * u;
    if (r >= r0 && r < K)
#pragma unroll
      for (int l = 0; l < kBand; ++l) bb.U()[(size_t)r * kBand + l] = Ur[u][l];
  }
}

// A22 -= V Y^T + Y V^T of panel p - 1 (p > 0) and the partial sums of
// X = A22 U of panel p (p < np) on a kTrailRows x kBandTile tile of the
// trailing matrix [8p + 8, K)^2 (both triangles).  Thread (row, quarter)
// takes 32 columns: all its loads are issued before any store (stores count
// against the same vector-memory counter as loads, so a load behind a store
// waits for it).  Four waves (one per SIMD) and at most 170 registers let
// three workgroups share a CU, so that one tile's loads overlap another's
// arithmetic.  X partials: one ld x kBand array per column tile.
constexpr int kTrailT = 256;
constexpr int kTrailRows = 64;
constexpr int kTrailQ = kTrailT / kTrailRows;         // column groups
constexpr int kTrailC = kBandTile / kTrailQ;          // columns per thread
template <bool ADMM>
__global__ __launch_bounds__(kTrailT, 3) void k_band_trail(LargeArgs a, int p) {
  __shared__ double cs[kBandTile][3 * kBand];   // V, Y, U of the tile's columns
  __shared__ double xh[kTrailQ - 1][kTrailRows][kBand];
  const int K = a.tsize[blockIdx.x];
  if (K < a.band_min) return;
  const int np = band_panels(K);
  if (p > np) return;
  const int R0 = p * kBand + kBand, n = K - R0;
  if (n <= 0) return;
  const int ntr = (n + kTrailRows - 1) / kTrailRows, ntc = (n + kBandTile - 1) / kBandTile;
  if ((int)blockIdx.y >= ntr * ntc) return;
  const int tr = blockIdx.y % ntr, tc = blockIdx.y / ntr;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int ld = lead_dim(K);
  const BandBufs bb = band_bufs(w, ld);
  double* W = w.W;
  const bool upd = p > 0, sym = p < np;
  const int vpar = (p + 1) & 1;   // V of panel p - 1
  const int tid = threadIdx.x;
  const int cb0 = R0 + tc * kBandTile;
  const int rl = tid & (kTrailRows - 1), qt = tid / kTrailRows;
  const int r = R0 + tr * kTrailRows + rl;
  const int rc = min(r, K - 1);
  const int cs0 = qt * kTrailC;                       // first tile column of this thread
  // the thread's 32 entries (clamped addresses), issued first
  double x[kTrailC];
#pragma unroll
  for (int j = 0; j < kTrailC; ++j) x[j] = W[(size_t)min(cb0 + cs0 + j, K - 1) * ld + rc];
  // column operands (offset arithmetic: V, U, Y are kBand ld-row arrays at
  // slots vpar, 2 and 3 of the workspace) and the row's V and Y, all loads
  // issued before the first LDS store
  constexpr int kCsN = kBandTile * 3 * kBand / kTrailT;
  static_assert(kCsN * kTrailT == kBandTile * 3 * kBand, "column operand staging");
  double cv[kCsN];
#pragma unroll
  for (int q = 0; q < kCsN; ++q) {
    const int idx = tid + kTrailT * q;
    const int cc = idx / (3 * kBand), f = idx - cc * (3 * kBand), c = min(cb0 + cc, K - 1);
    const int sel = (f < kBand) ? vpar : ((f < 2 * kBand) ? 3 : 2);
    const bool on = (f < 2 * kBand) ? upd : sym;
    cv[q] = on ? bb.S[(size_t)sel * kBand * ld + (size_t)c * kBand + (f & (kBand - 1))] : 0.0;
  }
  double vr[kBand], yr[kBand], acc[kBand];
#pragma unroll
  for (int l = 0; l < kBand; ++l) {
    vr[l] = upd ? bb.V(vpar)[(size_t)rc * kBand + l] : 0.0;
    yr[l] = upd ? bb.Y()[(size_t)rc * kBand + l] : 0.0;
    acc[l] = 0.0;
  }
#pragma unroll
  for (int q = 0; q < kCsN; ++q) {
    const int idx = tid + kTrailT * q;
    const int cc = idx / (3 * kBand), f = idx - cc * (3 * kBand);
    cs[cc][f] = cv[q];
  }
  __syncthreads();
  const int ncc = min(kTrailC, K - (cb0 + cs0));       // valid columns (may be <= 0)
  // (the empty asm statements keep the compiler from loading every
  // column's LDS operands into registers at once)
  if (upd) {
#pragma unroll
    for (int j = 0; j < kTrailC; ++j) {
      double t = x[j];
#pragma unroll
      for (int l = 0; l < kBand; ++l) t -= vr[l] * cs[cs0 + j][kBand + l] + yr[l] * cs[cs0 + j][l];
      x[j] = t;
      asm volatile("" ::: "memory");
    }
    if (r < K)
#pragma unroll
      for (int j = 0; j < kTrailC; ++j)
        if (j < ncc) W[(size_t)(cb0 + cs0 + j) * ld + r] = x[j];
  }
  if (sym) {
#pragma unroll
    for (int j = 0; j < kTrailC; ++j) {
      const double t = (j < ncc) ? x[j] : 0.0;
      double u8[kBand];
#pragma unroll
      for (int l = 0; l < kBand; ++l) u8[l] = cs[cs0 + j][2 * kBand + l];
#pragma unroll
      for (int l = 0; l < kBand; ++l) acc[l] += t * u8[l];
      asm volatile("" ::: "memory");
    }
    if (qt > 0)
#pragma unroll
      for (int l = 0; l < kBand; ++l) xh[qt - 1][rl][l] = acc[l];
    __syncthreads();
    if (qt == 0 && r < K)
#pragma unroll
      for (int l = 0; l < kBand; ++l) {
        double t = acc[l];
#pragma unroll
        for (int g = 0; g < kTrailQ - 1; ++g) t += xh[g][rl][l];
        bb.X()[((size_t)tc * ld + r) * kBand + l] = t;
      }
  }
}

// Stage 2: the band (diagonals 0..kBand of W) to tridiagonal form in LDS,
// one workgroup per task.  Stored diagonals: L[d][j] = B(j + d, j),
// d < 2 kBand (a bulge reaches 2 kBand - 1 below the diagonal); entries
// past the matrix are zero and stay zero (a step's rows and columns past K
// hold zeros in and out), so the steps need no bounds tests.  Step k of
// sweep s reads and writes C = B(r:r+8, r-8:r) and D = B(r:r+8, r:r+8),
// r = s + 1 + 8k: it must follow step k + 1 of sweep s - 1 (whose C
// overlaps D) and is disjoint from step k + 2 of sweep s - 1, so sweep s
// runs two steps behind sweep s - 1.
// An 8-lane group runs one sweep, lane i holding row i of the step's 8 x 8
// blocks (sums over a block's rows are 3 DPP exchanges, a reflector's
// 8-vector reaches the group's lanes through LDS, sums along a row stay in
// the lane).  A wave runs 8 consecutive sweeps in lockstep, group g
// 2 steps behind group g - 1 (wave step t is step t - 2 g of sweep base +
// g), which is the order the dependence needs; the first group waits on the
// previous wave's last sweep through an LDS progress flag
// (sweep * 256 + steps done, + 255 when the sweep ends).
constexpr int kChaseG = 8;                   // sweeps per wave

// sum over the lane's aligned group of 8 (every lane gets it)
__device__ __forceinline__ double sum8(double x) {
  x += dpp_f64<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += dpp_f64<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += dpp_f64<0x141>(x);   // row_half_mirror: lane j <-> 7 - j of the group
  return x;
}
template <bool ADMM>
__global__ __launch_bounds__(64 * kChaseWaves) void k_band_chase(LargeArgs a) {
  static_assert(kBand == 8 && kChaseG == 8, "one 8-lane group per sweep, 8 x 8 blocks");
  __shared__ double L[2 * kBand * kChaseLd];
  __shared__ int prog[kChaseWaves];
  __shared__ __align__(16) double vb[kChaseWaves][64];   // a group's 8-vector, gathered through LDS
  const int K = a.tsize[blockIdx.x];
  if (K < a.band_min) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int ld = lead_dim(K);
  const double* W = w.W;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int idx = tid; idx < 2 * kBand * kChaseLd; idx += 64 * kChaseWaves) {
    const int j = idx / (2 * kBand), d = idx - j * (2 * kBand);
    double x = 0.0;
    if (d <= kBand && j + d < K) x = W[(size_t)j * ld + j + d];
    L[d * kChaseLd + j] = x;
  }
  if (tid < kChaseWaves) prog[tid] = -1;
  __syncthreads();
  const int g = lane >> 3, i = lane & 7;
  const bool upper = (i & 4) != 0;
  const int NK = band_nk(K);
  const int pw = (wv + kChaseWaves - 1) % kChaseWaves;
  // Progress flags order LDS data only: a wave publishes after its LDS
  // accesses have completed (s_waitcnt lgkmcnt(0), not waiting for its
  // global stores of reflectors, which only later kernels read), and a
  // waiting wave reads the flag with a volatile load before its data loads
  // (LDS requests are served in order).
  volatile int* vprog = prog;
  bool fail = false;
  auto house = [](double alpha, double ss, double& beta, double& tu, double& scale) {
    if (ss == 0.0) {
      beta = alpha;
      tu = 0.0;
      scale = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + ss), alpha);
      tu = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
  };
  for (int base = wv * kChaseG; base < K - 2; base += kChaseWaves * kChaseG) {
    const int s = base + g;
    const int nst = (s < K - 2) ? (K - 1 - s + kBand - 1) / kBand : 0;   // steps of sweep s
    const int nst0 = (K - 1 - base + kBand - 1) / kBand;
    const int T = 2 * (kChaseG - 1) + nst0;                             // wave steps (group 0 is longest)
    double pv[kBand], ptu = 0.0;
#pragma unroll
    for (int q = 0; q < kBand; ++q) pv[q] = 0.0;
    for (int t = 0; t < T; ++t) {
      // group 0 (sweep base) may run step t once sweep base - 1 (the
      // previous wave's last group) has completed step t + 1
      if (base > 0 && !fail && t < nst0) {
        const int need = (base - 1) * 256 + min(t + 2, 255);
        int it = 0;
        while (vprog[pw] < need) {
          if (++it > kChaseSpin) {
            fail = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        asm volatile("" ::: "memory");
      }
      const int k = t - 2 * g;
      if (k >= 0 && k < nst) {
        // rows r.. of the block the step annihilates and reduces; the
        // previous reflector's column block r - 8.. (step 0: column s = r - 1)
        const int r = s + 1 + kBand * k;
        // C = B(r:r+8, r-8:r), row i: entry jj at diagonal 8 + i - jj,
        // column r - 8 + jj, i.e. (7 - jj) (kChaseLd - 1) after entry 7
        // (diagonal 1 + i, column r - 1), which at step 0 is column s, the
        // only column that step reads (every address stays inside L:
        // diagonals 1..15, columns >= r - 8 > -kChaseLd);
        // D = B(r:r+8, r:r+8), row i
        double* c7 = &L[(1 + i) * kChaseLd + r - 1];
        double c[kBand], dr[kBand];
#pragma unroll
        for (int jj = 0; jj < kBand; ++jj) {
          c[jj] = c7[(kBand - 1 - jj) * (kChaseLd - 1)];
          const int hi = max(i, jj), lo = min(i, jj);
          dr[jj] = L[(hi - lo) * kChaseLd + r + lo];
        }
        if (k == 0) {
          c[0] = c[kBand - 1];
#pragma unroll
          for (int jj = 1; jj < kBand; ++jj) c[jj] = 0.0;
        }
        if (k > 0) {
          // C <- C H_prev (the fill the previous reflector makes)
          double t1 = 0.0;
#pragma unroll
          for (int jj = 0; jj < kBand; ++jj) t1 += c[jj] * pv[jj];
#pragma unroll
          for (int jj = 0; jj < kBand; ++jj) c[jj] -= ptu * t1 * pv[jj];
        }
        // the reflector of C's first column: H C(:, 0) = beta e_1
        const double x = c[0];
        const double ss = sum8((i >= 1) ? x * x : 0.0);
        double beta, tu, scale;
        double alpha;   // x of lane 0 of the group
        {
          const double y0 = dpp_f64<0x00>(x), z0 = dpp_f64<0x141>(y0);
          alpha = upper ? z0 : y0;
        }
        house(alpha, ss, beta, tu, scale);
        const double vi = (i == 0) ? 1.0 : x * scale;
        // v of the group to every lane: through the wave's LDS row (one
        // wave, its LDS accesses in order)
        double v[kBand];
        vb[wv][lane] = vi;
#pragma unroll
        for (int q = 0; q < kBand; ++q) v[q] = vb[wv][(lane & ~7) + q];
        // C <- H C (the first column exactly beta e_1)
#pragma unroll
        for (int jj = 1; jj < kBand; ++jj) {
          const double u = sum8(vi * c[jj]);
          c[jj] -= tu * vi * u;
        }
        c[0] = (i == 0) ? beta : 0.0;
        if (k > 0) {
#pragma unroll
          for (int jj = 0; jj < kBand; ++jj) c7[(kBand - 1 - jj) * (kChaseLd - 1)] = c[jj];
        } else {
          c7[0] = c[0];
        }
        w.refl[((size_t)s * NK + k) * kBandRefl + i] = (i == 0) ? tu : vi;
        // D <- H D H: p = tau D v, w = p - tau/2 (p^T v) v, D -= v w^T + w v^T
        double p = 0.0;
#pragma unroll
        for (int jj = 0; jj < kBand; ++jj) p += dr[jj] * v[jj];
        p *= tu;
        const double pvs = sum8(p * vi);
        const double wi = p - 0.5 * tu * pvs * vi;
        double wa[kBand];
        vb[wv][lane] = wi;
#pragma unroll
        for (int q = 0; q < kBand; ++q) wa[q] = vb[wv][(lane & ~7) + q];
#pragma unroll
        for (int jj = 0; jj < kBand; ++jj) dr[jj] -= vi * wa[jj] + wi * v[jj];
#pragma unroll
        for (int jj = 0; jj < kBand; ++jj)
          if (jj <= i) L[(i - jj) * kChaseLd + r + jj] = dr[jj];
#pragma unroll
        for (int q = 0; q < kBand; ++q) pv[q] = v[q];
        ptu = tu;
      }
      // publish the progress of the last group's sweep
      const int sl = base + kChaseG - 1, kl = t - 2 * (kChaseG - 1) + 1;
      const int nstl = (K - 1 - sl + kBand - 1) / kBand;
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's LDS accesses done
      asm volatile("" ::: "memory");
      if (lane == 0) vprog[wv] = sl * 256 + ((kl >= nstl) ? 255 : max(kl, 0));
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);
    asm volatile("" ::: "memory");
    if (lane == 0) vprog[wv] = (base + kChaseG - 1) * 256 + 255;
  }
  __syncthreads();
  if (fail && lane == 0) w.meta[5] = 1.0;
  for (int j = tid; j < K; j += 64 * kChaseWaves) {
    w.d[j] = L[j];
    w.e[j] = (j < K - 1) ? L[kChaseLd + j] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// 3. eigenpairs of T on the smaller-signed side
// ---------------------------------------------------------------------------
// 1 / q for normal q with |q| < 2^1022: the hardware reciprocal estimate
// (relative error ~5e-8) and two Newton steps, which round exactly as 1.0 / q
// does on every sample tested over the exponent range; about half the
// dependent latency of the full division sequence
__device__ __forceinline__ double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return fma(r, fma(-q, r, 1.0), r);
}

__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int K, double x, double pivmin) {
  // number of eigenvalues of T smaller than x (LDL^T signs of T - x I);
  // |q| >= pivmin keeps q normal and e2 / q finite
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int i = 1; i < K; ++i) {
    q = (d[i] - x) - e2[i - 1] * rcp_nr(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

// LU of T - lambda I with partial pivoting (T tridiagonal: diagonal d,
// off-diagonal e).  Row i of U holds (U0, U1, U2) on columns i, i+1, i+2;
// stored: L multiplier, pivot flag, 1 / U0, U1, U2, arrays a = 0..4 at
// f[a * KR + i * st].  Pivots below tiny are raised to +-tiny.
__device__ __forceinline__ void tri_factor(const double* d, const double* e, int K, double lam, double tiny,
                                           double* f, int st, size_t KR) {
  double al = d[0] - lam, be = (K > 1) ? e[0] : 0.0;
  for (int i = 0; i < K - 1; ++i) {
    const double cc = e[i], an = d[i + 1] - lam, bn = (i + 1 < K - 1) ? e[i + 1] : 0.0;
    const bool piv = fabs(al) < fabs(cc);
    double a0 = al;
    if (!piv && fabs(a0) < tiny) a0 = (a0 < 0.0) ? -tiny : tiny;
    const double u0 = piv ? cc : a0;
    const double au = fabs(u0);
    const double r0 = (au > 1e-290 && au < 1e290) ? rcp_nr(u0) : 1.0 / u0;
    const double l = (piv ? al : cc) * r0;
    const size_t o = (size_t)i * st;
    f[o] = l;
    f[KR + o] = piv ? 1.0 : 0.0;
    f[2 * KR + o] = r0;
    f[3 * KR + o] = piv ? an : be;
    f[4 * KR + o] = piv ? bn : 0.0;
    const double nal = piv ? (be - l * an) : (an - l * be);
    const double nbe = piv ? (-l * bn) : bn;
    al = nal;
    be = nbe;
  }
  if (fabs(al) < tiny) al = (al < 0.0) ? -tiny : tiny;
  const size_t o = (size_t)(K - 1) * st;
  f[o] = 0.0;
  f[KR + o] = 0.0;
  f[2 * KR + o] = 1.0 / al;
  f[3 * KR + o] = 0.0;
  f[4 * KR + o] = 0.0;
}

// One inverse-iteration solve (T - lambda I) z_new = sc * z in place (z at
// stride zs); returns 1 / ||z_new||.  Both sweeps are recurrences carried in
// registers; the operands of C consecutive steps are loaded ahead (clamped
// indices, no predicated loads) so that one lane's chain does not wait on
// every load.
template <int C>
__device__ __forceinline__ double tri_solve(const double* __restrict__ f, int st, size_t KR, int K, double* z,
                                            int zs, double sc, double* zo = nullptr, int zos = 0) {
  if (!zo) {
    zo = z;
    zos = zs;
  }
  // forward: P and the unit lower bidiagonal L
  double cur = z[0] * sc;
  for (int i0 = 0; i0 < K - 1; i0 += C) {
    double raw[C], lv[C], pv[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int i = min(i0 + j, K - 2);
      raw[j] = z[(size_t)(i + 1) * zs];
      lv[j] = f[(size_t)i * st];
      pv[j] = f[KR + (size_t)i * st];
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int i = i0 + j;
      if (i < K - 1) {
        const double rw = raw[j] * sc;
        const bool p = pv[j] != 0.0;
        const double out = p ? rw : cur;
        const double oth = p ? cur : rw;
        z[(size_t)i * zs] = out;
        cur = oth - lv[j] * out;
      }
    }
  }
  z[(size_t)(K - 1) * zs] = cur;
  // backward: upper triangular with two superdiagonals
  double z1 = 0.0, z2 = 0.0, nn = 0.0;
  for (int i0 = K - 1; i0 >= 0; i0 -= C) {
    double zv[C], u1[C], u2[C], r0[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const size_t o = (size_t)max(i0 - j, 0);
      zv[j] = z[o * zs];
      u1[j] = f[3 * KR + o * st];
      u2[j] = f[4 * KR + o * st];
      r0[j] = f[2 * KR + o * st];
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int i = i0 - j;
      if (i >= 0) {
        const double zi = (zv[j] - u1[j] * z1 - u2[j] * z2) * r0[j];
        zo[(size_t)i * zos] = zi;
        nn += zi * zi;
        z2 = z1;
        z1 = zi;
      }
    }
  }
  return 1.0 / sqrt(nn);
}

// tri_solve for factors and iterate in global memory: the same arithmetic in
// the same order, with the operands of the next C steps loaded while the
// current C are processed (two register sets), so that a sweep waits for
// memory once instead of once per C steps
template <int C>
__device__ __forceinline__ double tri_solve_pf(const double* __restrict__ f, int st, size_t KR, int K, double* z,
                                               int zs, double sc, double* zo = nullptr, int zos = 0) {
  if (!zo) {
    zo = z;
    zos = zs;
  }
  // forward: P and the unit lower bidiagonal L (elements 0 .. K - 2; the
  // loads of a batch read z above the rows the earlier batches write)
  double cur = z[0] * sc;
  auto fload = [&](int i0, double (&raw)[C], double (&lv)[C], double (&pv)[C]) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int i = min(i0 + j, K - 2);
      raw[j] = z[(size_t)(i + 1) * zs];
      lv[j] = f[(size_t)i * st];
      pv[j] = f[KR + (size_t)i * st];
    }
  };
  auto fproc = [&](int i0, const double (&raw)[C], const double (&lv)[C], const double (&pv)[C]) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int i = i0 + j;
      if (i < K - 1) {
        const double rw = raw[j] * sc;
        const bool p = pv[j] != 0.0;
        const double out = p ? rw : cur;
        const double oth = p ? cur : rw;
        z[(size_t)i * zs] = out;
        cur = oth - lv[j] * out;
      }
    }
  };
  {
    double ra[C], la[C], pa[C], rb[C], lb[C], pb[C];
    fload(0, ra, la, pa);
    for (int i0 = 0; i0 < K - 1; i0 += 2 * C) {
      fload(i0 + C, rb, lb, pb);
      fproc(i0, ra, la, pa);
      fload(i0 + 2 * C, ra, la, pa);
      fproc(i0 + C, rb, lb, pb);
    }
  }
  z[(size_t)(K - 1) * zs] = cur;
  // backward: upper triangular with two superdiagonals (rows K - 1 .. 0; the
  // loads of a batch read rows below those the earlier batches write)
  double z1 = 0.0, z2 = 0.0, nn = 0.0;
  auto bload = [&](int i0, double (&zv)[C], double (&u1)[C], double (&u2)[C], double (&r0)[C]) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const size_t o = (size_t)max(i0 - j, 0);
      zv[j] = z[o * zs];
      u1[j] = f[3 * KR + o * st];
      u2[j] = f[4 * KR + o * st];
      r0[j] = f[2 * KR + o * st];
    }
  };
  auto bproc = [&](int i0, const double (&zv)[C], const double (&u1)[C], const double (&u2)[C], const double (&r0)[C]) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int i = i0 - j;
      if (i >= 0) {
        const double zi = (zv[j] - u1[j] * z1 - u2[j] * z2) * r0[j];
        zo[(size_t)i * zos] = zi;
        nn += zi * zi;
        z2 = z1;
        z1 = zi;
      }
    }
  };
  {
    double za[C], ua[C], va[C], ra[C], zb[C], ub[C], vb[C], rb[C];
    bload(K - 1, za, ua, va, ra);
    for (int i0 = K - 1; i0 >= 0; i0 -= 2 * C) {
      bload(i0 - C, zb, ub, vb, rb);
      bproc(i0, za, ua, va, ra);
      bload(i0 - 2 * C, za, ua, va, ra);
      bproc(i0 - C, zb, ub, vb, rb);
    }
  }
  return 1.0 / sqrt(nn);
}

// (a) prep, one workgroup per task: negligible off-diagonals are set to zero
//     (they split T), the Gershgorin bound, the Sturm count at 0 and the
//     side; meta = [r, pos, first, pivmin, ||T||]
template <bool ADMM>
__global__ __launch_bounds__(kLT) void k_eig_prep(LargeArgs a) {
  __shared__ double sd[1024], se[1024];
  __shared__ double se2[1024];
  __shared__ double red[kLT / 64 + 1];
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int tid = threadIdx.x;
  for (int i = tid; i < K; i += kLT) {
    sd[i] = w.d[i];
    se[i] = (i < K - 1) ? w.e[i] : 0.0;
  }
  __syncthreads();
  double tn = 0.0;
  for (int i = tid; i < K; i += kLT) {
    const double em = (i > 0) ? fabs(se[i - 1]) : 0.0;
    tn = fmax(tn, fabs(sd[i]) + em + fabs(se[i]));
  }
  for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_xor(tn, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = tn;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int q = 0; q < kLT / 64; ++q) m = fmax(m, red[q]);
    red[kLT / 64] = m;
  }
  __syncthreads();
  tn = red[kLT / 64];
  __syncthreads();
  double emax2 = 0.0;
  for (int i = tid; i < K - 1; i += kLT) {
    double ei = se[i];
    if (fabs(ei) <= kEps * (fabs(sd[i]) + fabs(sd[i + 1]))) ei = 0.0;
    w.e[i] = ei;
    se2[i] = ei * ei;
    emax2 = fmax(emax2, ei * ei);
  }
  for (int off = 32; off > 0; off >>= 1) emax2 = fmax(emax2, __shfl_xor(emax2, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = emax2;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int q = 0; q < kLT / 64; ++q) m = fmax(m, red[q]);
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, m) / kEps;
    const int nneg = sturm_count(sd, se2, K, 0.0, pivmin);
    const int pos = (nneg <= K - nneg) ? 0 : 1;
    w.meta[0] = (double)(pos ? K - nneg : nneg);   // r
    w.meta[1] = (double)pos;
    w.meta[2] = (double)(pos ? nneg : 0);           // index of the first chosen eigenvalue
    w.meta[3] = pivmin;
    w.meta[4] = fmax(tn, 2.2250738585072014e-308);
  }
}

// (b) bisection: a group of kBisL lanes per eigenvalue (4 per wave, 16 per
//     workgroup of 4 waves).  The group's lanes evaluate the Sturm count at
//     kBisL interior points (multisection) and the interval shrinks by
//     kBisL + 1 per round; 16 points take 13 rounds where 64 take 9, for a
//     quarter of the lanes.  The chosen side lies in [Gershgorin low, 0] or
//     [0, Gershgorin high]; the count at 0 is the nneg of the prep, so
//     count(lo) <= k < count(hi) holds from the start.  Intervals are refined
//     to an absolute width of about eps ||T||, the accuracy inverse iteration
//     and the low-rank update can use.
constexpr int kBisL = 16;
constexpr int kBisWaves = 4;
constexpr int kBisEig = kBisWaves * (64 / kBisL);
template <bool ADMM>
__global__ __launch_bounds__(64 * kBisWaves) void k_eig_bisect(LargeArgs a) {
  __shared__ double sd[1024], se2[1024];
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int r = (int)w.meta[0];
  const int t0 = blockIdx.y * kBisEig;
  if (t0 >= r) return;
  const int pos = (int)w.meta[1], first = (int)w.meta[2];
  const double pivmin = w.meta[3], tnorm = w.meta[4];
  const int tid = threadIdx.x, lane = tid & 63, grp = lane / kBisL, gl = lane % kBisL;
  const int t = t0 + (tid >> 6) * (64 / kBisL) + grp;
  for (int i = tid; i < K; i += 64 * kBisWaves) {
    sd[i] = w.d[i];
    const double ei = (i < K - 1) ? w.e[i] : 0.0;
    se2[i] = ei * ei;
  }
  __syncthreads();
  if (t0 + (tid >> 6) * (64 / kBisL) >= r) return;   // whole waves; no barriers below
  const bool act = t < r;
  const double glo = -tnorm * (1.0 + 4.0 * kEps) - pivmin, ghi = tnorm * (1.0 + 4.0 * kEps) + pivmin;
  const double wtol = 2.0 * kEps * tnorm + 4.0 * pivmin;
  const int k = first + t;
  double lo = pos ? 0.0 : glo, hi = pos ? ghi : 0.0;
  for (int round = 0; round < 200; ++round) {
    const double width = hi - lo;
    const bool done = !act || width <= fmax(wtol, 2.0 * kEps * fmax(fabs(lo), fabs(hi)));
    if (__ballot(!done) == 0) break;
    const double step = width / (double)(kBisL + 1);
    const double x = lo + step * (double)(gl + 1);
    const uint64_t m = __ballot(!done && sturm_count(sd, se2, K, x, pivmin) > k);
    const uint32_t gm = (uint32_t)((m >> (grp * kBisL)) & ((1ull << kBisL) - 1ull));
    const int j0 = gm ? __builtin_ctz(gm) : kBisL;   // first point with count > k
    if (!done) {
      const double nlo = (j0 == 0) ? lo : lo + step * (double)j0;
      const double nhi = (j0 == kBisL) ? hi : lo + step * (double)(j0 + 1);
      lo = nlo;
      hi = fmax(nhi, nlo);
    }
  }
  if (act && gl == 0) w.lam[t] = 0.5 * (lo + hi);
}

// Inverse iteration with a partially pivoted LU of T - lambda I.  The
// factors of eigenvalue t live in the scratch area element-major (entry i of
// array a at ((a * K + i) * r + t)), so lanes that work on consecutive
// eigenvalues touch consecutive addresses; 6 K r <= 3 K^2 since r <= K / 2.
// Eigenvalues closer than 1e-5 ||T|| to a neighbour form clusters.
__device__ __forceinline__ double eig_ortol(double tnorm) { return 1e-5 * tnorm; }

// (c) isolated eigenvalues: kSingle per workgroup, one lane each, with the
//     LU factors and the iterate of each in LDS (6 K doubles per eigenvalue),
//     so the sequential sweeps never wait on global memory; two solves, the
//     second writing the eigenvector straight into its column of Z (its
//     normalisation is applied by the back-transformation).  Two solves
//     suffice: lambda is accurate to ~eps ||T|| and its gap to the other
//     eigenvalues is above 1e-5 ||T||, so each solve shrinks the other
//     components of a random start by ~1e-10 or more.
//     The LDS-resident form (kSingle eigenvalues of orders up to kSingleK,
//     54 KB per workgroup) suits small tasks with few chosen eigenvalues; the
//     others use the wide form below (64 eigenvalues per workgroup, factors
//     in the element-major global scratch), whose lanes are all busy.  (The
//     LDS form sized for order 1024 held one workgroup of two busy lanes per
//     CU: 364 us per max-cut iteration at its start, where every task has at
//     most 32 chosen eigenvalues.)
constexpr int kSingle = 8;
constexpr int kSingleLds = 32;
constexpr int kSingleK = 136;
__device__ __forceinline__ bool single_lds(int r, int K) { return r <= kSingleLds && K <= kSingleK; }
template <bool ADMM>
__global__ __launch_bounds__(64) void k_eig_single(LargeArgs a) {
  __shared__ double sd[kSingleK], se[kSingleK];
  __shared__ double F[kSingle][6 * kSingleK];
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int r = (int)w.meta[0];
  if (!single_lds(r, K) || blockIdx.y * kSingle >= r) return;
  const double tnorm = w.meta[4];
  for (int i = threadIdx.x; i < K; i += 64) {
    sd[i] = w.d[i];
    se[i] = (i < K - 1) ? w.e[i] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.y * kSingle + threadIdx.x;
  if (threadIdx.x >= kSingle || t >= r) return;
  const double lam = w.lam[t], ortol = eig_ortol(tnorm);
  const bool iso = (t == 0 || lam - w.lam[t - 1] > ortol) && (t == r - 1 || w.lam[t + 1] - lam > ortol);
  if (!iso) return;
  double* f = F[threadIdx.x];    // arrays a = 0..4 at f[a K + i], the iterate at f[5 K + i]
  double* z = f + 5 * K;
  tri_factor(sd, se, K, lam, kEps * tnorm, f, 1, (size_t)K);
  for (int i = 0; i < K; ++i) z[i] = hash_unit((uint32_t)t, (uint32_t)i);
  double sc = tri_solve<8>(f, 1, (size_t)K, K, z, 1, 1.0);
  sc = tri_solve<8>(f, 1, (size_t)K, K, z, 1, sc, w.Z + (size_t)t * K, 1);
  w.zs[t] = sc;
}

template <bool ADMM>
__global__ __launch_bounds__(64) void k_eig_single_wide(LargeArgs a) {
  __shared__ double sd[1024], se[1024];
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int r = (int)w.meta[0];
  if (single_lds(r, K) || blockIdx.y * 64 >= r) return;
  const double tnorm = w.meta[4];
  for (int i = threadIdx.x; i < K; i += 64) {
    sd[i] = w.d[i];
    se[i] = (i < K - 1) ? w.e[i] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.y * 64 + threadIdx.x;
  if (t >= r) return;
  const double lam = w.lam[t], ortol = eig_ortol(tnorm);
  const bool iso = (t == 0 || lam - w.lam[t - 1] > ortol) && (t == r - 1 || w.lam[t + 1] - lam > ortol);
  if (!iso) return;
  // element-major scratch: entry i of array a of eigenvalue t at (a K + i) r + t
  double* X = w.S;
  const size_t KR = (size_t)K * r;
  double* zt = X + 5 * KR + t;
  tri_factor(sd, se, K, lam, kEps * tnorm, X + t, r, KR);
  for (int i = 0; i < K; ++i) zt[(size_t)i * r] = hash_unit((uint32_t)t, (uint32_t)i);
  double sc = tri_solve_pf<16>(X + t, r, KR, K, zt, r, 1.0);
  sc = tri_solve_pf<16>(X + t, r, KR, K, zt, r, sc, w.Z + (size_t)t * K, 1);
  w.zs[t] = sc;
}

// (d) eigenvectors of the clustered eigenvalues (the isolated ones are (c)):
//     one 64-lane workgroup per cluster (the c-th run of eigenvalues whose
//     consecutive gaps are at most 1e-5 ||T||, found by a scan of lam).
//     Each member's factorisation of T - lambda I, start vector and first
//     solve depend on no other member: they run first, one lane per member,
//     on the element-major scratch of the wide form.  Then the members are
//     taken in order: factors and iterate are copied to LDS, and three times
//     the wave orthogonalises the iterate against the cluster's finished
//     members (classical Gram-Schmidt, twice) and normalises it, with lane 0's
//     sequential solves in between.  The finished vector goes to its column of
//     Z (scale 1).
template <bool ADMM>
__global__ __launch_bounds__(64) void k_eig_cluster(LargeArgs a) {
  __shared__ double sd[1024], se[1024];
  __shared__ double F[6 * 1024];
  __shared__ double slam[512];
  __shared__ double sdot[512];
  __shared__ int span[2];
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int r = (int)w.meta[0];
  if ((int)blockIdx.y * 2 >= r) return;   // a cluster has at least 2 members
  const int lane = threadIdx.x;
  const double tnorm = w.meta[4], ortol = eig_ortol(tnorm);
  for (int t = lane; t < r; t += 64) slam[t] = w.lam[t];
  __syncthreads();
  if (lane == 0) {
    // start and end of the blockIdx.y-th cluster of size >= 2
    int c = -1, t0 = 0, found0 = -1, found1 = -1;
    for (int t = 1; t <= r; ++t) {
      if (t == r || slam[t] - slam[t - 1] > ortol) {
        if (t - t0 >= 2 && ++c == (int)blockIdx.y) {
          found0 = t0;
          found1 = t;
          break;
        }
        t0 = t;
      }
    }
    span[0] = found0;
    span[1] = found1;
  }
  for (int i = lane; i < K; i += 64) {
    sd[i] = w.d[i];
    se[i] = (i < K - 1) ? w.e[i] : 0.0;
  }
  __syncthreads();
  const int c0 = span[0], c1 = span[1];
  if (c0 < 0) return;
  const double tiny = kEps * tnorm;
  // (i) per member, one lane each: factors, start vector, first solve
  //     (entry i of array a of member t at (a K + i) r + t; a = 5: iterate)
  double* X = w.S;
  const size_t KR = (size_t)K * r;
  for (int t = c0 + lane; t < c1; t += 64) {
    tri_factor(sd, se, K, slam[t], tiny, X + t, r, KR);
    double* zt = X + 5 * KR + t;
    for (int i = 0; i < K; ++i) zt[(size_t)i * r] = hash_unit((uint32_t)t, (uint32_t)i);
    (void)tri_solve_pf<16>(X + t, r, KR, K, zt, r, 1.0);
  }
  __syncthreads();
  // (ii) members in order
  double* f = F;              // LU arrays a = 0..4 at f[a K + i]
  double* z = F + 5 * K;      // the member's iterate
  for (int t = c0; t < c1; ++t) {
    for (int idx = lane; idx < 6 * K; idx += 64) F[idx] = X[(size_t)idx * r + t];
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      if (it > 0) {
        if (lane == 0) (void)tri_solve<8>(f, 1, (size_t)K, K, z, 1, 1.0);
        __syncthreads();
      }
      // classical Gram-Schmidt applied twice against the cluster's finished
      // members: all their dot products with z first (16 at a time, loads in
      // flight together), then one update, instead of one dependent
      // dot-and-update round per member
      for (int pass = 0; pass < 2; ++pass) {
        for (int p0 = c0; p0 < t; p0 += 16) {
          const int np = min(16, t - p0);
          double dots[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) dots[u] = 0.0;
          for (int i = lane; i < K; i += 64) {
            const double zi = z[i];
#pragma unroll
            for (int u = 0; u < 16; ++u) dots[u] += w.Z[(size_t)(p0 + min(u, np - 1)) * K + i] * zi;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const double s = wave_sum(dots[u]);
            if (lane == 0 && u < np) sdot[p0 - c0 + u] = s;
          }
        }
        __syncthreads();
        for (int i = lane; i < K; i += 64) {
          double acc = 0.0;
          for (int p = c0; p < t; ++p) acc += sdot[p - c0] * w.Z[(size_t)p * K + i];
          z[i] -= acc;
        }
        __syncthreads();
      }
      double nn = 0.0;
      for (int i = lane; i < K; i += 64) nn += z[i] * z[i];
      const double sc = 1.0 / sqrt(wave_sum(nn));
      for (int i = lane; i < K; i += 64) z[i] *= sc;
      __syncthreads();
    }
    double* zo = w.Z + (size_t)t * K;
    for (int i = lane; i < K; i += 64) zo[i] = z[i];
    if (lane == 0) w.zs[t] = 1.0;
    __threadfence_block();
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 4. back-transformation V = Q Z = H_0 H_1 ... H_{K-3} Z, blocked: the
//    reflectors of panel p (columns j0 = 32 p ..) form
//    B_p = H_j0 ... H_j0+31 = I - V_p T_p V_p^T with T_p upper triangular
//    (the compact WY form, Schreiber & Van Loan; T(i,i) = tau_i,
//    T(0:i, i) = -tau_i T(0:i, 0:i) V_p(:, 0:i)^T v_i), and
//    Q Z = B_0 (B_1 (... B_{P-1} Z)).
// ---------------------------------------------------------------------------
// Z <- Q2 Z for the tasks of the two-stage reduction, Q2 the product of the
// bulge-chasing reflectors in the order they were made: sweeps from the last
// to the first (a sweep's reflectors act on disjoint rows s + 1 + kBand k
// onwards and commute).  One wave per kQ2C eigenvectors, held in LDS row by
// row; lane (k, c) applies reflector k (+ 64 / kQ2C per pass) of the sweep to
// eigenvector c.  The next sweep's reflectors are loaded into registers
// while the current sweep runs and stored over them after it (one wave:
// LDS accesses are served in order, no barrier).
constexpr int kQ2C = 4;
// reflector passes whose loads are issued together (1 against 2, 3, 4 and 8:
// 1.61, 1.69, 1.74, 1.78 and 2.48 ms per max-cut iteration; fewer registers)
constexpr int kQ2Pass = 1;
template <bool ADMM>
__global__ __launch_bounds__(64) void k_band_q2(LargeArgs a) {
  // rows of the eigenvectors, (kmax + kBand) x kQ2C doubles sized at launch
  // (rows past K stay zero): with the reflector buffer 30 KB at order 673,
  // five workgroups per CU
  extern __shared__ double Zr[];
  __shared__ double R[128 * kBandRefl];   // the current sweep's reflectors
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  if (K < a.band_min) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int r = (int)w.meta[0];
  const int c0 = blockIdx.y * kQ2C;
  if (c0 >= r) return;
  const int nc = min(kQ2C, r - c0);
  constexpr int kQ2K = 64 / kQ2C;   // reflectors per pass
  const int lane = threadIdx.x, c = lane & (kQ2C - 1), kk = lane / kQ2C;
  const int NK = band_nk(K);
  // the eigenvectors into LDS, 8 loads in flight per lane (clamped
  // addresses, the value selected after)
  for (int i0 = 0; i0 < kQ2C * (K + kBand); i0 += 64 * 8) {
    double zv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = i0 + lane + 64 * q, row = idx / kQ2C, cl = idx - row * kQ2C;
      zv[q] = w.Z[(size_t)(c0 + min(cl, nc - 1)) * K + min(row, K - 1)];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = i0 + lane + 64 * q;
      const int row = idx / kQ2C, cl = idx - row * kQ2C;
      if (row < K + kBand) Zr[idx] = (cl < nc && row < K) ? zv[q] : 0.0;
    }
  }
  constexpr int kPre = 128 * kBandRefl / 64;   // reflector doubles per lane per sweep
  auto nsteps = [&](int s) { return (K - 1 - s + kBand - 1) / kBand; };
  auto load_sweep = [&](int s, double (&x)[kPre]) {
    const double* src = w.refl + (size_t)s * NK * kBandRefl;
    const int n = nsteps(s) * kBandRefl;
#pragma unroll
    for (int q = 0; q < kPre; ++q) x[q] = src[min(lane + 64 * q, n - 1)];
  };
  double x[kPre];
  load_sweep(K - 3, x);
#pragma unroll
  for (int q = 0; q < kPre; ++q) R[lane + 64 * q] = x[q];
  for (int s = K - 3; s >= 0; --s) {
    if (s > 0) load_sweep(s - 1, x);   // in registers until this sweep is done
    const double* rs_ = R;
    const int ns = nsteps(s);
    // passes of kQ2K reflectors (lane (k, c): reflector kk + kQ2K j), kQ2Pass at
    // a time: all their loads first (the passes touch disjoint rows), then
    // the updates.  Reflector entries past the matrix are stored as zero.
    for (int j0 = 0; kQ2K * j0 < ns; j0 += kQ2Pass) {
      double z[kQ2Pass][kBand], v[kQ2Pass][kBand];
      int rsq[kQ2Pass];
#pragma unroll
      for (int jq = 0; jq < kQ2Pass; ++jq) {
        const int k = kk + kQ2K * (j0 + jq);
        const bool on = k < ns;
        rsq[jq] = on ? s + 1 + kBand * k : K;   // K: a zero row block
        const double* rf = rs_ + min(k, NK - 1) * kBandRefl;
#pragma unroll
        for (int i = 0; i < kBand; ++i) {
          z[jq][i] = Zr[(rsq[jq] + i) * kQ2C + c];
          v[jq][i] = on ? ((i == 0) ? 1.0 : rf[i]) : 0.0;
        }
        rsq[jq] = on ? rsq[jq] : -1;
        const double tu = on ? rf[0] : 0.0;   // the record's slot 0 holds tau (v_0 = 1)
        double dot = 0.0;
#pragma unroll
        for (int i = 0; i < kBand; ++i) dot += v[jq][i] * z[jq][i];
        dot *= tu;
#pragma unroll
        for (int i = 0; i < kBand; ++i) z[jq][i] -= dot * v[jq][i];
      }
#pragma unroll
      for (int jq = 0; jq < kQ2Pass; ++jq)
        if (rsq[jq] >= 0)
#pragma unroll
          for (int i = 0; i < kBand; ++i) Zr[(rsq[jq] + i) * kQ2C + c] = z[jq][i];
    }
    if (s > 0)
#pragma unroll
      for (int q = 0; q < kPre; ++q) R[lane + 64 * q] = x[q];
  }
  for (int idx = lane; idx < nc * K; idx += 64) {
    const int cl = idx / K, row = idx - cl * K;
    w.Z[(size_t)(c0 + cl) * K + row] = Zr[row * kQ2C + cl];
  }
}

constexpr int kBtNC = 8;     // eigenvectors per apply workgroup, resident in LDS
constexpr int kBtCR = 128;   // rows of a staged V panel chunk (1.01 -> 0.97 ms per max-cut iteration against 256)

// element (row, a) of V_p: the reflector of column c = j0 + a has 1 on row
// c + sh and the stored Householder vector below it (sh = 1 after the
// one-stage reduction, kBand after the dense-to-band stage, whose column c
// keeps the band on rows c..c+kBand)
__device__ __forceinline__ double bt_v(const double* W, int ld, int K, int j0, int nbp, int a, int row, int sh) {
  if (a >= nbp || row >= K || row < j0 + a + sh) return 0.0;
  return (row == j0 + a + sh) ? 1.0 : W[(size_t)(j0 + a) * ld + row];
}

// reflector columns of a task: 0 .. bt_ncols - 1
__device__ __forceinline__ int bt_ncols(int K, int sh) { return K - 1 - sh; }

__device__ __forceinline__ double* bt_tbuf(const Ws& w) { return w.S; }   // 32 x 32 per panel

// Stage rows [row0, row0 + kBtCR) of the panel's 32 reflectors into Vc, in
// two parts: bt_fetch issues the loads into registers, bt_put stores the
// values (so that the next chunk's loads can be in flight while the current
// one is used).  Every load is unconditional, from a clamped address inside
// the task's W (column j0 + min(a, nbp - 1) <= K - 3, row <= K - 1), and the
// empty asm statements take each loaded value as an operand, so the compiler
// cannot move a load under its lane condition: the thread's loads are in
// flight together instead of one round trip each.  The value is selected
// when it is stored.
constexpr int kBtNQ = kBtCR * 32 / 1024;
__device__ __forceinline__ void bt_fetch(double (&x)[kBtNQ], const double* W, int ld, int K, int j0, int nbp, int row0,
                                         int tid) {
#pragma unroll
  for (int q = 0; q < kBtNQ; ++q) {
    const int idx = tid + 1024 * q, as = idx / kBtCR, rl = idx - as * kBtCR;
    x[q] = W[(size_t)(j0 + min(as, nbp - 1)) * ld + min(row0 + rl, K - 1)];
  }
#pragma unroll
  for (int q = 0; q < kBtNQ; ++q) asm volatile("" : "+v"(x[q]));
}
__device__ __forceinline__ void bt_put(double (*Vc)[33], const double (&x)[kBtNQ], int K, int j0, int nbp, int row0,
                                       int tid, int sh) {
#pragma unroll
  for (int q = 0; q < kBtNQ; ++q) {
    const int idx = tid + 1024 * q, as = idx / kBtCR, rl = idx - as * kBtCR, row = row0 + rl;
    const bool zero = as >= nbp || row >= K || row < j0 + as + sh;
    Vc[rl][as] = zero ? 0.0 : ((row == j0 + as + sh) ? 1.0 : x[q]);
  }
}
template <bool ADMM>
__global__ __launch_bounds__(1024) void k_bt_tfactor(LargeArgs a) {
  __shared__ double Vc[32][33];
  __shared__ double G[32][33];
  __shared__ double Ts[32][33];
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  const int sh = (K >= a.band_min) ? kBand : 1;
  const int ncols = bt_ncols(K, sh);
  const int P = (ncols + kNB - 1) / kNB;
  const int p = blockIdx.y;
  if (p >= P) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  if ((int)w.meta[0] == 0) return;
  const int ld = lead_dim(K);
  const int j0 = p * kNB, nbp = min(kNB, ncols - j0);
  const int tid = threadIdx.x, ta = tid >> 5, tb = tid & 31;
  // Gram matrix V_p^T V_p over 32-row chunks staged in LDS
  double g = 0.0;
  for (int row0 = j0 + sh; row0 < K; row0 += 32) {
    Vc[tb][ta] = bt_v(w.W, ld, K, j0, nbp, ta, row0 + tb, sh);   // Vc[row][col]
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < 32; ++rr) g += Vc[rr][ta] * Vc[rr][tb];
    __syncthreads();
  }
  G[ta][tb] = g;
  __syncthreads();
  if (tid < 64) {
    const int k = tid;
    for (int i = 0; i < kNB; ++i) {
      const double tu = (i < nbp) ? w.tau[j0 + i] : 0.0;
      double t = 0.0;
      if (k < i)
        for (int m = k; m < i; ++m) t += Ts[k][m] * G[m][i];
      if (k < 32) Ts[k][i] = (k < i) ? -tu * t : ((k == i) ? tu : 0.0);
    }
  }
  __syncthreads();
  bt_tbuf(w)[(size_t)p * kNB * kNB + ta * kNB + tb] = Ts[ta][tb];
}

template <bool ADMM>
__global__ __launch_bounds__(1024) void k_bt_apply(LargeArgs a) {
  __shared__ double Zs[kBtNC][1024];
  __shared__ double Vc[kBtCR][33];
  __shared__ double Sp[4][32][kBtNC];
  __shared__ double Sq[32][kBtNC];
  __shared__ double Ts[32][33];
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int r = (int)w.meta[0];
  const int c0 = blockIdx.y * kBtNC;
  if (c0 >= r) return;
  const int nc = min(kBtNC, r - c0);
  const int ld = lead_dim(K);
  const int sh = (K >= a.band_min) ? kBand : 1;   // Q2 already applied by k_band_q2
  const int ncols = bt_ncols(K, sh);
  const int P = (ncols + kNB - 1) / kNB;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kBtNC * K; idx += 1024) {
    const int cl = idx / K, row = idx - cl * K;
    Zs[cl][row] = (cl < nc) ? w.Z[(size_t)(c0 + cl) * K + row] * w.zs[c0 + cl] : 0.0;
  }
  const int a1 = tid & 31, cl1 = (tid >> 5) & 7, h1 = tid >> 8;   // pass 1: S(a, cl), row phase h
  const int rl3 = tid & 127, cl3 = tid >> 7;                        // pass 2: Z(row, cl)
  // Chunks in order: panels P-1 .. 0, each pass 1 then pass 2 over rows
  // [j0 + sh, K) in steps of kBtCR; the next chunk's reflectors (and the next
  // panel's T) are loaded while the current chunk is used.
  auto jb = [&](int p) { return p * kNB; };
  auto nb = [&](int p) { return min(kNB, ncols - p * kNB); };
  double x[kBtNQ];
  bt_fetch(x, w.W, ld, K, jb(P - 1), nb(P - 1), jb(P - 1) + sh, tid);
  double tnext = bt_tbuf(w)[(size_t)(P - 1) * kNB * kNB + tid];
  for (int p = P - 1; p >= 0; --p) {
    const int j0 = jb(p), nbp = nb(p);
    Ts[tid >> 5][tid & 31] = tnext;
    if (p > 0) tnext = bt_tbuf(w)[(size_t)(p - 1) * kNB * kNB + tid];
    double sp = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      for (int row0 = j0 + sh; row0 < K; row0 += kBtCR) {
        bt_put(Vc, x, K, j0, nbp, row0, tid, sh);
        __syncthreads();
        // the chunk after this one
        if (row0 + kBtCR < K) {
          bt_fetch(x, w.W, ld, K, j0, nbp, row0 + kBtCR, tid);
        } else if (pass == 0) {
          bt_fetch(x, w.W, ld, K, j0, nbp, j0 + sh, tid);
        } else if (p > 0) {
          bt_fetch(x, w.W, ld, K, jb(p - 1), nb(p - 1), jb(p - 1) + sh, tid);
        }
        const int nr = min(kBtCR, K - row0);
        if (pass == 0) {
          // pass 1: S = V_p^T Z
          for (int rr = h1; rr < nr; rr += 4) sp += Vc[rr][a1] * Zs[cl1][row0 + rr];
        } else {
          // pass 2: Z -= V_p S
#pragma unroll
          for (int hh = 0; hh < kBtCR / 128; ++hh) {
            const int rr = hh * 128 + rl3, row = row0 + rr;
            if (row < K) {
              double t = 0.0;
#pragma unroll 8
              for (int aa = 0; aa < 32; ++aa) t += Vc[rr][aa] * Sq[aa][cl3];
              Zs[cl3][row] -= t;
            }
          }
        }
        __syncthreads();
      }
      if (pass == 0) {
        Sp[h1][a1][cl1] = sp;
        __syncthreads();
        // S <- T S
        if (tid < 32 * kBtNC) {
          const int k = tid & 31, cl = tid >> 5;
          double t = 0.0;
          for (int m = k; m < 32; ++m) t += Ts[k][m] * ((Sp[0][m][cl] + Sp[1][m][cl]) + (Sp[2][m][cl] + Sp[3][m][cl]));
          Sq[k][cl] = t;
        }
        __syncthreads();
      }
    }
  }
  for (int idx = tid; idx < nc * K; idx += 1024) {
    const int cl = idx / K, row = idx - cl * K;
    w.Z[(size_t)(c0 + cl) * K + row] = Zs[cl][row];
  }
}

// ---------------------------------------------------------------------------
// 5. reconstruction tiles + fused dual update
// ---------------------------------------------------------------------------
template <bool ADMM>
__global__ __launch_bounds__(256) void k_large_recon(LargeArgs a) {
  __shared__ double Va[kTile][kTile + 1];
  __shared__ double Vb[kTile][kTile + 1];
  __shared__ double red[256 / 64 + 1];
  int K;
  int64_t base;
  if (!task_info<ADMM>(a, blockIdx.x, K, base)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int T = (K + kTile - 1) / kTile;
  const int ntile = T * (T + 1) / 2;
  const int q = blockIdx.y;
  if (q >= ntile) return;
  int ti = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > q) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= q) ++ti;
  const int tj = q - ti * (ti + 1) / 2;
  const int a0 = ti * kTile, b0 = tj * kTile;
  const int r = (int)w.meta[0], pos = (int)w.meta[1];
  const int tid = threadIdx.x;
  const int ty = tid / 8, tx = tid % 8;          // 32 rows x (8 threads x 4 columns)
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  constexpr int NI = kTile * kTile / 256;
  static_assert(NI * 256 == kTile * kTile, "recon staging");
  for (int l0 = 0; l0 < r; l0 += kTile) {
    // every load from a clamped in-range address (column <= r - 1 < K,
    // row <= K - 1), issued together; the empty asm statements keep the
    // compiler from moving them under their lane conditions
    double za[NI], zb[NI], lm[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int idx = tid + 256 * q, ii = idx % kTile, l = min(l0 + idx / kTile, r - 1);
      const double* zl = w.Z + (size_t)l * K;
      za[q] = zl[min(a0 + ii, K - 1)];
      zb[q] = zl[min(b0 + ii, K - 1)];
      lm[q] = w.lam[l];
    }
#pragma unroll
    for (int q = 0; q < NI; ++q) asm volatile("" : "+v"(za[q]), "+v"(zb[q]), "+v"(lm[q]));
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int idx = tid + 256 * q, ii = idx % kTile, ll = idx / kTile;
      const bool lv = l0 + ll < r;
      Va[ii][ll] = (lv && a0 + ii < K) ? za[q] * lm[q] : 0.0;
      Vb[ii][ll] = (lv && b0 + ii < K) ? zb[q] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ll = 0; ll < kTile; ++ll) {
      const double x = Va[ty][ll];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += x * Vb[tx * 4 + u][ll];
    }
    __syncthreads();
  }
  double ex = 0.0, ev = 0.0;
  const int ai = a0 + ty;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int bi = b0 + tx * 4 + u;
    if (ai < K && bi < K && ai >= bi) {
      const int t = packed_index(ai, bi, K);
      const double sc = (ai == bi) ? 1.0 : kSqrt2;
      const double y = yvec_of<ADMM>(a, base, t);
      const double sp = pos ? acc[u] * sc : y - acc[u] * sc;
      if (ADMM) {
        const int64_t sl = base + t;
        const double sv = a.d.s[sl], zv = a.d.z[sl], vv = a.d.v[sl];
        const int e = a.d.slot2ent[sl];
        const double xh = a.d.xh[e];
        const double xv = a.d.relax ? a.d.x[e] : xh;   // (H x+) at the slot
        const double zn = sp - y;
        const double vn = slot_vnew(a.d, sv, zv, vv, xh);
        a.d.s[sl] = sp;
        a.d.z[sl] = zn;
        a.d.v[sl] = vn;
        ex += (xv - sp) * (xv - sp);
        ev += (vn - zn) * (vn - zn);
      } else {
        a.pout[base + t] = sp;
      }
    }
  }
  if (ADMM) {
    ex = block_sum<256>(ex, red);
    ev = block_sum<256>(ev, red);
    if (tid == 0) {
      w.tiles[2 * q] = ex;
      w.tiles[2 * q + 1] = ev;
    }
  }
}

__global__ __launch_bounds__(64) void k_large_partials(LargeArgs a) {
  int K;
  int64_t base;
  if (!task_info<true>(a, blockIdx.x, K, base)) return;
  Ws w = ws_of(a.work + a.woff[blockIdx.x], K);
  const int T = (K + kTile - 1) / kTile;
  const int ntile = T * (T + 1) / 2;
  double ex = 0.0, ev = 0.0;
  for (int q = threadIdx.x; q < ntile; q += 64) {
    ex += w.tiles[2 * q];
    ev += w.tiles[2 * q + 1];
  }
  ex = wave_sum(ex);
  ev = wave_sum(ev);
  if (threadIdx.x == 0) {
    const int k = a.tasks[blockIdx.x];
    a.d.part_c[2 * k] = ex;
    a.d.part_c[2 * k + 1] = ev;
  }
}

template <bool ADMM>
static void run_large_step(const LargeArgs& a, int32_t ntask, int32_t kmax, const int32_t* host_sizes, int step,
                           hipStream_t st, const LaunchHook* hook = nullptr) {
  if (ntask <= 0) return;
  const int rmax = kmax / 2 + 1;
  const int T = (kmax + kTile - 1) / kTile;
  auto launch_shm = [&](int kind, auto kernel, dim3 grid, dim3 block, size_t shm, auto... args) {
    if (hook) {
      hipEvent_t e0, e1;
      hook->begin(hook->ctx, kind, &e0, &e1);
      hipExtLaunchKernelGGL(kernel, grid, block, shm, st, e0, e1, 0, args...);
      hook->end(hook->ctx, kind);
    } else {
      hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
    }
  };
  auto launch = [&](int kind, auto kernel, dim3 grid, dim3 block, auto... args) {
    launch_shm(kind, kernel, grid, block, 0, args...);
  };
  switch (step) {
    case 0: hipLaunchKernelGGL(k_large_gather<ADMM>, dim3(ntask, T * (T + 1) / 2), dim3(256), 0, st, a); break;
    case 1: {
      // tasks are sorted by order (descending): the two-stage tasks (order
      // >= band_min) form a prefix, and so do the tasks that still have a
      // given panel
      int nband = 0;
      while (nband < ntask && host_sizes[nband] >= a.band_min) ++nband;
      if (nband) {
        const int npm = band_panels(host_sizes[0]);
        for (int p = 0; p <= npm; ++p) {
          int na = 0;
          while (na < nband && band_panels(host_sizes[na]) >= p) ++na;
          launch(10, k_band_panel<ADMM>, dim3(na), dim3(kBandT), a, p);
          const int n = host_sizes[0] - p * kBand - kBand;
          if (n > 0) {
            const int ntr = (n + kTrailRows - 1) / kTrailRows, ntc = (n + kBandTile - 1) / kBandTile;
            launch(11, k_band_trail<ADMM>, dim3(na, ntr * ntc), dim3(kTrailT), a, p);
          }
        }
        launch(12, k_band_chase<ADMM>, dim3(nband), dim3(64 * kChaseWaves), a);
      }
      // one-stage: the panel steps of the remaining tasks in lockstep, then
      // one launch finishes every such task in LDS
      auto active = [&](int j0) {
        int n = 0;
        while (n < ntask && trd_tail_start(host_sizes[n]) > j0) ++n;
        return n;
      };
      if (nband == ntask) break;
      const int kmax1 = host_sizes[nband];   // largest one-stage order
      const int np = trd_tail_start(kmax1) / kNB;
      const int ldm = (kmax1 + 7) & ~7;
      for (int p = 0; p < np; ++p) {
        const int na = active(p * kNB);
        for (int i = 0; i < kNB; ++i) {
          const int j = p * kNB + i;
          const int nallm = kmax1 - j - 1 + 2 * i;
          const int ncy = (nallm + kSymvCols - 1) / kSymvCols;
          const int nrbm = (ldm - ((j + 1) & ~1) + kSymvRows - 1) / kSymvRows;
          launch(0, k_trd_symv<ADMM>, dim3(na, ncy * nrbm), dim3(256), a, p, i, ncy);
          launch(1, k_trd_update<ADMM>, dim3(na, (ldm + kUpdRows - 1) / kUpdRows), dim3(256), a, p, i);
        }
        const int n2 = kmax1 - p * kNB - kNB;
        launch(2, k_trd_trail<ADMM>, dim3(na, ((n2 + 127) / 128) * ((n2 + 63) / 64)), dim3(kTT), a, p);
      }
      // the smaller tail shape when every one-stage clique fits it
      if (kmax1 <= 64)
        launch(3, k_trd_tail<ADMM, 64, 256, 64>, dim3(ntask), dim3(256), a);
      else
        launch(3, k_trd_tail<ADMM, kTail, 1024, 144>, dim3(ntask), dim3(1024), a);
      break;
    }
    case 2:
      launch(4, k_eig_prep<ADMM>, dim3(ntask), dim3(kLT), a);
      launch(5, k_eig_bisect<ADMM>, dim3(ntask, (rmax + kBisEig - 1) / kBisEig), dim3(64 * kBisWaves), a);
      launch(6, k_eig_single<ADMM>, dim3(ntask, (std::min(rmax, kSingleLds) + kSingle - 1) / kSingle), dim3(64), a);
      launch(6, k_eig_single_wide<ADMM>, dim3(ntask, (rmax + 63) / 64), dim3(64), a);
      launch(7, k_eig_cluster<ADMM>, dim3(ntask, (rmax + 1) / 2), dim3(64), a);
      break;
    case 3:
      if (host_sizes[0] >= a.band_min) {
        // dynamic LDS above 64 KB (orders above 1000) needs the kernel's
        // limit raised; set once per process
        static const bool raised = [] {
          const int bytes = (1024 + kBand) * kQ2C * (int)sizeof(double);
          return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_band_q2<ADMM>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
        }();
        (void)raised;
        launch_shm(13, k_band_q2<ADMM>, dim3(ntask, (rmax + kQ2C - 1) / kQ2C), dim3(64),
                   (size_t)(kmax + kBand) * kQ2C * sizeof(double), a);
      }
      launch(8, k_bt_tfactor<ADMM>, dim3(ntask, (kmax - 2 + kNB - 1) / kNB), dim3(1024), a);
      launch(9, k_bt_apply<ADMM>, dim3(ntask, (rmax + kBtNC - 1) / kBtNC), dim3(1024), a);
      break;
    case 4: hipLaunchKernelGGL(k_large_recon<ADMM>, dim3(ntask, T * (T + 1) / 2), dim3(256), 0, st, a); break;
    case 5:
      if (ADMM) hipLaunchKernelGGL(k_large_partials, dim3(ntask), dim3(64), 0, st, a);
      break;
    default: break;
  }
}

void launch_cone_large_step(const DevPlan& d, const int32_t* tasks, int32_t ntask, int32_t kmax,
                            const int32_t* host_sizes, int step, hipStream_t st, int band_min,
                            const LaunchHook* hook) {
  LargeArgs a{};
  a.d = d;
  a.tasks = tasks;
  a.work = d.big_work;
  a.woff = d.big_off;
  a.tsize = d.big_size;
  a.band_min = band_min;
  run_large_step<true>(a, ntask, kmax, host_sizes, step, st, hook);
}

void launch_psd_project_large(const int32_t* sizes, const int64_t* offs, const int32_t* tasks,
                              const int32_t* task_sizes, const int32_t* host_sizes, int32_t ntask, int32_t kmax,
                              const double* in, double* out, double* work, const int64_t* work_off, hipStream_t st,
                              int band_min) {
  LargeArgs a{};
  a.band_min = band_min;
  a.tasks = tasks;
  a.psizes = sizes;
  a.poffs = offs;
  a.pin = in;
  a.pout = out;
  a.work = work;
  a.woff = work_off;
  a.tsize = task_sizes;
  for (int step = 0; step < kLargeSteps; ++step) run_large_step<false>(a, ntask, kmax, host_sizes, step, st);
}

}  // namespace cdcs
