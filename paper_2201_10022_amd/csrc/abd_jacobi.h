// Register-resident cyclic Jacobi eigen-solver and PSD projection for small
// symmetric matrices (one matrix per lane).
//
// The matrix is kept packed (upper triangle, N(N+1)/2 doubles) and the
// eigenvector matrix V (N*N doubles) in registers; all loops over (p,q) and
// rows are fully unrolled so every index is a compile-time constant and no
// register array is indexed dynamically.  Each rotation zeroes A(p,q) with
// the symmetric 2x2 Schur decomposition (Golub & Van Loan, sec. 8.5), using
// t = sgn(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp, which
// needs no guard against huge d / a_pq ratios; lanes whose matrix has already
// converged execute identity rotations (t = 0) to keep the wave uniform.
#pragma once
#include <hip/hip_runtime.h>

// true when the predicate holds on every lane of the wave (host builds of
// the same arithmetic, used for checking, see a single lane)
__host__ __device__ __forceinline__ bool wave_all(bool p) {
#ifdef __HIP_DEVICE_COMPILE__
  return __all(p);
#else
  return p;
#endif
}

template <int N>
struct SymIdx {
  static constexpr int at(int i, int j) {
    return i <= j ? i * N - (i * (i - 1)) / 2 + (j - i) : j * N - (j * (j - 1)) / 2 + (i - j);
  }
};

template <int N, int P, int Q>
__host__ __device__ __forceinline__ void jacobi_rotate(double *A, double *V) {
  using S = SymIdx<N>;
  const double apq = A[S::at(P, Q)];
  const double app = A[S::at(P, P)];
  const double aqq = A[S::at(Q, Q)];
  const double d = aqq - app;
  const double den = fabs(d) + sqrt(d * d + 4.0 * apq * apq);
  double t = den > 0.0 ? 2.0 * apq / den : 0.0;
  t = d < 0.0 ? -t : t;
  const double c = 1.0 / sqrt(t * t + 1.0);
  const double s = t * c;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k == P || k == Q) continue;
    const double akp = A[S::at(k, P)], akq = A[S::at(k, Q)];
    A[S::at(k, P)] = c * akp - s * akq;
    A[S::at(k, Q)] = s * akp + c * akq;
  }
  A[S::at(P, P)] = app - t * apq;
  A[S::at(Q, Q)] = aqq + t * apq;
  A[S::at(P, Q)] = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double vkp = V[k * N + P], vkq = V[k * N + Q];
    V[k * N + P] = c * vkp - s * vkq;
    V[k * N + Q] = s * vkp + c * vkq;
  }
}

template <int N, int P, int Q>
struct JacobiSweep {
  static __host__ __device__ __forceinline__ void run(double *A, double *V) {
    jacobi_rotate<N, P, Q>(A, V);
    if constexpr (Q + 1 < N)
      JacobiSweep<N, P, Q + 1>::run(A, V);
    else if constexpr (P + 2 < N)
      JacobiSweep<N, P + 1, P + 2>::run(A, V);
  }
};

// Eigen-decomposition: on return A's diagonal holds the eigenvalues and V's
// columns the eigenvectors.  Stops when every lane's off-diagonal mass is
// below rel_tol^2 of its Frobenius mass, or after max_sweeps.
template <int N>
__host__ __device__ __forceinline__ int jacobi_eig(double *A, double *V, int max_sweeps, double rel_tol2) {
  using S = SymIdx<N>;
#pragma unroll
  for (int i = 0; i < N * N; ++i) V[i] = (i % (N + 1) == 0) ? 1.0 : 0.0;
  double frob = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) frob += (i == j ? 1.0 : 2.0) * A[S::at(i, j)] * A[S::at(i, j)];
  int sweeps = 0;
  for (; sweeps < max_sweeps; ++sweeps) {
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += A[S::at(i, j)] * A[S::at(i, j)];
    const bool done = !(off > rel_tol2 * frob);
    if (wave_all(done)) break;
    JacobiSweep<N, 0, 1>::run(A, V);
  }
  return sweeps;
}

// A <- sum_{lambda_k > 0} lambda_k v_k v_k^T (packed), i.e. the nearest PSD
// matrix in the Frobenius norm.
template <int N>
__host__ __device__ __forceinline__ void psd_project_packed(double *A) {
  using S = SymIdx<N>;
  double V[N * N];
  jacobi_eig<N>(A, V, 30, 1e-32);
  double lam[N];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = fmax(A[S::at(k, k)], 0.0);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += lam[k] * V[i * N + k] * V[j * N + k];
      A[S::at(i, j)] = acc;
    }
}
