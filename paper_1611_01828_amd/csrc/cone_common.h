// Device routines shared by the cone kernels and the adjoint kernels: packed
// (svec) block indexing, the symmetric 2x2 Schur rotation and cyclic Jacobi
// with round-robin parallel ordering on a block held in LDS (Golub & Van
// Loan, Matrix Computations, Sections 8.5.2-8.5.5).
#pragma once

#include "device.h"

namespace cdcs {

namespace jac {

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

// Symmetric Schur 2x2: (c, s, t) with t = tan(theta) annihilating A_pq, in
// the working precision T (above `big`, 1 + theta^2 would overflow and
// t = 1 / (2 theta) to working accuracy).
template <typename T>
__device__ __forceinline__ void schur2(T app, T aqq, T apq, T& c, T& s, T& t) {
  if (apq == T(0)) {
    c = T(1);
    s = T(0);
    t = T(0);
    return;
  }
  const T big = sizeof(T) == 8 ? T(1e150) : T(1e18);
  const T theta = (aqq - app) / (T(2) * apq);
  const T at = fabs(theta);
  T tt;
  if (at > big) {
    tt = T(0.5) / theta;
  } else {
    tt = T(1) / (at + sqrt(T(1) + at * at));
    if (theta < T(0)) tt = -tt;
  }
  c = T(1) / sqrt(T(1) + tt * tt);
  s = tt * c;
  t = tt;
}

}  // namespace jac

using namespace jac;

template <typename T>
struct Pair2;
template <>
struct Pair2<double> { using type = double2; };
template <>
struct Pair2<float> { using type = float2; };

// The rotations of one round, one per disjoint pair: (c, s) together and
// p | q << 16 in one word, so that a work item reads each pair's rotation
// with two LDS loads.
template <int KMAX, typename T>
struct JacRot {
  typename Pair2<T>::type cs[KMAX / 2];
  T t[KMAX / 2];      // tan(theta), for the 2x2 diagonal blocks
  int pq[KMAX / 2];
};

// Cyclic Jacobi on the KP x KP (KP even, zero padded) matrix in LDS, in the
// working precision T (double, or float for the FP32 variant; the
// convergence sums are kept in double).  On return A holds the eigenvalues
// on its diagonal and V the eigenvectors.
template <int KMAX, int NT, typename T = double>
__device__ void jacobi_lds(T* A, T* V, int K, int KP, JacRot<KMAX, T>& rot, double* red) {
  const int tid = threadIdx.x;
  const int half = KP / 2;
  // The work items of a round, idx = tid + NT u split as (idx / half,
  // idx % half), are stepped without a division: (a0, b0) for u = 0 and
  // (sa, sb) per step, computed once.
  const int a0 = tid / half, b0 = tid - a0 * half;
  const int sa = NT / half, sb = NT - sa * half;
  // off(A)^2 <= tol ||A||_F^2: (1e-16)^2 in FP64; in FP32 a little above
  // (2^-23)^2 so that rounding cannot keep the sweeps going
  const double tol = sizeof(T) == 8 ? 1e-32 : 1e-13;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = tid; idx < K * K; idx += NT) {
      const int i = idx / K, j = idx - (idx / K) * K;
      const double a = (double)A[i * KMAX + j];
      tot += a * a;
      if (i != j) off += a * a;
    }
    off = block_sum<NT>(off, red);
    tot = block_sum<NT>(tot, red);
    if (!(off > tol * tot)) break;   // also stops on 0 or NaN
    // round-robin positions (tid + r) mod (KP - 1) and (KP - 1 - tid + r)
    // mod (KP - 1), stepped once per round
    int pm = tid % (KP - 1), qm = (KP - 1 - tid) % (KP - 1);
    for (int r = 0; r < KP - 1; ++r) {
      if (tid < half) {
        int p, q;
        if (tid == 0) {
          p = 0;
          q = 1 + pm;   // r mod (KP - 1)
        } else {
          p = 1 + pm;
          q = 1 + qm;
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        T c, s, t;
        schur2<T>(A[p * KMAX + p], A[q * KMAX + q], A[p * KMAX + q], c, s, t);
        rot.pq[tid] = p | (q << 16);
        rot.cs[tid].x = c;
        rot.cs[tid].y = s;
        rot.t[tid] = t;
      }
      pm = (pm + 1 == KP - 1) ? 0 : pm + 1;
      qm = (qm + 1 == KP - 1) ? 0 : qm + 1;
      __syncthreads();
      // A <- J^T A J on disjoint 2x2 blocks; V <- V J (neighbouring work
      // items share the row pair and walk along rows of A and V)
      for (int idx = tid, a = a0, bq = b0; idx < half * half;
           idx += NT, a += sa + (bq + sb >= half), bq += sb - (bq + sb >= half ? half : 0)) {
        const int pqa = rot.pq[a], pqb = rot.pq[bq];
        const int pa = pqa & 0xffff, qa = pqa >> 16, pb = pqb & 0xffff, qb = pqb >> 16;
        if (a == bq) {
          const T t = rot.t[a];
          const T apq = A[pa * KMAX + qa];
          A[pa * KMAX + pa] -= t * apq;
          A[qa * KMAX + qa] += t * apq;
          A[pa * KMAX + qa] = T(0);
          A[qa * KMAX + pa] = T(0);
        } else {
          const auto ra = rot.cs[a], rb = rot.cs[bq];
          const T ca = ra.x, sa_ = ra.y, cb = rb.x, sb_ = rb.y;
          const T x00 = A[pa * KMAX + pb], x01 = A[pa * KMAX + qb];
          const T x10 = A[qa * KMAX + pb], x11 = A[qa * KMAX + qb];
          const T y00 = ca * x00 - sa_ * x10, y01 = ca * x01 - sa_ * x11;
          const T y10 = sa_ * x00 + ca * x10, y11 = sa_ * x01 + ca * x11;
          A[pa * KMAX + pb] = y00 * cb - y01 * sb_;
          A[pa * KMAX + qb] = y00 * sb_ + y01 * cb;
          A[qa * KMAX + pb] = y10 * cb - y11 * sb_;
          A[qa * KMAX + qb] = y10 * sb_ + y11 * cb;
        }
      }
      for (int idx = tid, i = a0, bq = b0; idx < KP * half;
           idx += NT, i += sa + (bq + sb >= half), bq += sb - (bq + sb >= half ? half : 0)) {
        const int pqb = rot.pq[bq];
        const int pb = pqb & 0xffff, qb = pqb >> 16;
        const auto rb = rot.cs[bq];
        const T cb = rb.x, sb_ = rb.y;
        const T vp = V[i * KMAX + pb], vq = V[i * KMAX + qb];
        V[i * KMAX + pb] = cb * vp - sb_ * vq;
        V[i * KMAX + qb] = sb_ * vp + cb * vq;
      }
      __syncthreads();
    }
  }
}

// A <- V^T A V on the leading K x K blocks in LDS (warm start of the Jacobi
// iteration from the eigenvectors V of a nearby matrix), then symmetrised.
// Each thread keeps its entries of a product in registers until all threads
// have read the operand it overwrites.
template <int KMAX, int NT, typename T>
__device__ void similarity_lds(T* A, const T* V, int K) {
  constexpr int NO = (KMAX * KMAX + NT - 1) / NT;
  const int tid = threadIdx.x;
  T acc[NO];
  // A V
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int idx = tid + o * NT;
    if (idx < K * K) {
      const int i = idx / K, j = idx - (idx / K) * K;
      T sum = T(0);
      for (int l = 0; l < K; ++l) sum += A[i * KMAX + l] * V[l * KMAX + j];
      acc[o] = sum;
    }
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int idx = tid + o * NT;
    if (idx < K * K) A[(idx / K) * KMAX + idx - (idx / K) * K] = acc[o];
  }
  __syncthreads();
  // V^T (A V)
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int idx = tid + o * NT;
    if (idx < K * K) {
      const int i = idx / K, j = idx - (idx / K) * K;
      T sum = T(0);
      for (int l = 0; l < K; ++l) sum += V[l * KMAX + i] * A[l * KMAX + j];
      acc[o] = sum;
    }
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int idx = tid + o * NT;
    if (idx < K * K) A[(idx / K) * KMAX + idx - (idx / K) * K] = acc[o];
  }
  __syncthreads();
  // (B + B^T) / 2: the thread of (i, j), i < j, writes both
  for (int idx = tid; idx < K * K; idx += NT) {
    const int i = idx / K, j = idx - (idx / K) * K;
    if (i < j) {
      const T m = T(0.5) * (A[i * KMAX + j] + A[j * KMAX + i]);
      A[i * KMAX + j] = m;
      A[j * KMAX + i] = m;
    }
  }
  __syncthreads();
}

// V <- V (3 I - V^T V) / 2 on the leading K x K block (one Newton-Schulz
// step towards the nearest orthogonal matrix: an orthogonality error e
// becomes O(e^2)).  G is K x K scratch in LDS.
template <int KMAX, int NT, typename T>
__device__ void orthonormalize_lds(T* V, T* G, int K) {
  constexpr int NO = (KMAX * KMAX + NT - 1) / NT;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < K * K; idx += NT) {
    const int i = idx / K, j = idx - (idx / K) * K;
    T sum = T(0);
    for (int l = 0; l < K; ++l) sum += V[l * KMAX + i] * V[l * KMAX + j];
    G[i * KMAX + j] = sum;
  }
  __syncthreads();
  T acc[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int idx = tid + o * NT;
    if (idx < K * K) {
      const int i = idx / K, j = idx - (idx / K) * K;
      T sum = T(0);
      for (int l = 0; l < K; ++l) sum += V[i * KMAX + l] * G[l * KMAX + j];
      acc[o] = T(1.5) * V[i * KMAX + j] - T(0.5) * sum;
    }
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int idx = tid + o * NT;
    if (idx < K * K) V[(idx / K) * KMAX + idx - (idx / K) * K] = acc[o];
  }
  __syncthreads();
}

// Select the cheaper side of the spectrum: Pi_+(Y) = sum_{l>0} lam_l v v^T
// = Y - sum_{l<0} lam_l v v^T.  Fills sel[0..nsel) and returns sign flag
// (1 = positive side).  Runs on thread 0 only; result broadcast via LDS.
template <int NT, typename T = double>
__device__ void choose_side(const T* A, int K, int KMAX_, int* sel, int* meta) {
  if (threadIdx.x == 0) {
    int npos = 0;
    for (int l = 0; l < K; ++l) npos += (A[l * KMAX_ + l] > T(0));
    const int pos = (npos <= K - npos) ? 1 : 0;
    int n = 0;
    for (int l = 0; l < K; ++l) {
      const T lam = A[l * KMAX_ + l];
      if (pos ? (lam > T(0)) : (lam < T(0))) sel[n++] = l;
    }
    meta[0] = n;
    meta[1] = pos;
  }
  __syncthreads();
}


}  // namespace cdcs
