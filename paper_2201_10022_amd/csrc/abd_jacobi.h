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
//
// A sweep visits the N(N-1)/2 index pairs in the round-robin (parallel)
// order of Brent and Luk: each round holds floor(N/2) rotations on disjoint
// index pairs.  Rotations on disjoint pairs commute and none changes the 2x2
// block another one reads, so a round's angles all come from the matrix as
// the round starts; one lane then works on several independent sqrt/divide
// chains at once instead of one long dependent chain per sweep.
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

// angle of the rotation that zeroes A(P,Q): t = tan, c = cos, s = sin
template <int N, int P, int Q>
__host__ __device__ __forceinline__ void jacobi_angle(const double *A, double &t, double &c, double &s) {
  using S = SymIdx<N>;
  const double apq = A[S::at(P, Q)];
  const double d = A[S::at(Q, Q)] - A[S::at(P, P)];
  // den >= 2|a_pq|; the floor only matters for an all-zero 2x2 block,
  // where it gives t = 0 without a branch
  const double den = fmax(fabs(d) + sqrt(d * d + 4.0 * apq * apq), 1e-300);
  t = (d < 0.0 ? -2.0 : 2.0) * apq / den;
  c = 1.0 / sqrt(t * t + 1.0);
  s = t * c;
}

// A <- J^T A J, V <- V J for the rotation J on (P,Q) with the given angle
template <int N, int P, int Q>
__host__ __device__ __forceinline__ void jacobi_apply(double *A, double *V, double t, double c, double s) {
  using S = SymIdx<N>;
  const double apq = A[S::at(P, Q)];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k == P || k == Q) continue;
    const double akp = A[S::at(k, P)], akq = A[S::at(k, Q)];
    A[S::at(k, P)] = c * akp - s * akq;
    A[S::at(k, Q)] = s * akp + c * akq;
  }
  A[S::at(P, P)] -= t * apq;
  A[S::at(Q, Q)] += t * apq;
  A[S::at(P, Q)] = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double vkp = V[k * N + P], vkq = V[k * N + Q];
    V[k * N + P] = c * vkp - s * vkq;
    V[k * N + Q] = s * vkp + c * vkq;
  }
}

// K-th index pair of round R of the round-robin schedule: the players
// 0..M-1 (M = N for odd N, N-1 for even N) sit on a circle, player N (odd
// N: nobody) or N-1 (even N) is fixed; in round R, player R meets the fixed
// one and (R+k) meets (R-k) mod M for k >= 1.  Over M rounds every pair
// meets once.
template <int N, int R, int K>
struct RoundPair {
  static constexpr int M = N % 2 ? N : N - 1;
  static constexpr int KK = N % 2 ? K + 1 : K;  // odd N: the fixed player's partner idles
  static constexpr int a = KK == 0 ? R : (R + KK) % M;
  static constexpr int b = KK == 0 ? N - 1 : (R - KK + M) % M;
  static constexpr int P = a < b ? a : b;
  static constexpr int Q = a < b ? b : a;
};

template <int N, int R, int K>
__host__ __device__ __forceinline__ void round_angles(const double *A, double *t, double *c, double *s) {
  using RP = RoundPair<N, R, K>;
  jacobi_angle<N, RP::P, RP::Q>(A, t[K], c[K], s[K]);
  if constexpr (K + 1 < N / 2) round_angles<N, R, K + 1>(A, t, c, s);
}

template <int N, int R, int K>
__host__ __device__ __forceinline__ void round_apply(double *A, double *V, const double *t, const double *c,
                                                     const double *s) {
  using RP = RoundPair<N, R, K>;
  jacobi_apply<N, RP::P, RP::Q>(A, V, t[K], c[K], s[K]);
  if constexpr (K + 1 < N / 2) round_apply<N, R, K + 1>(A, V, t, c, s);
}

template <int N, int R>
struct JacobiSweep {
  static __host__ __device__ __forceinline__ void run(double *A, double *V) {
    double t[N / 2], c[N / 2], s[N / 2];
    round_angles<N, R, 0>(A, t, c, s);
    round_apply<N, R, 0>(A, V, t, c, s);
    if constexpr (R + 1 < RoundPair<N, 0, 0>::M) JacobiSweep<N, R + 1>::run(A, V);
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
    JacobiSweep<N, 0>::run(A, V);
  }
  return sweeps;
}

// A <- sum_{lambda_k > 0} lambda_k v_k v_k^T (packed), i.e. the nearest PSD
// matrix in the Frobenius norm.  Sweeps stop once the off-diagonal mass is
// below 1e-24 of the Frobenius mass: an error of about 1e-12 of the matrix
// in the projection (eigenvector components mixed across the sign change
// of the spectrum are weighted by the eigenvalue gap), a sweep sooner than
// at full precision.
template <int N>
__host__ __device__ __forceinline__ void psd_project_packed(double *A) {
  using S = SymIdx<N>;
  double V[N * N];
  jacobi_eig<N>(A, V, 30, 1e-24);
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
