// HIP kernels of the EMU quasi-Newton iteration (gfx950, wave64).
//
// One iteration of the method (Sec. 3.2.1, Algorithm 1) is the kernel sequence
//   element -> gram -> gram_reduce -> control_a -> uz -> direction
//   -> rhs -> forward levels -> backward levels -> lscoef -> control_b -> add_q
// Every kernel first reads ctl->done and returns when it is set, so a fixed
// sequence of many iterations can be replayed from a HIP graph and stop on the
// device.  All sums are deterministic: each workgroup reduces a fixed set of
// elements in a fixed tree order (double-double for energies, gradient norms
// and line-search coefficients), and a single workgroup adds the partials in
// workgroup order.  There are no floating-point atomics.
//
// Per-element variables: F_i = R_i S_i with R_i a rotation and S_i symmetric.
// The quasi-Newton step is taken in the rotated frame dF = R dX, with dX split
// into its symmetric (6) and skew (3) parts in orthonormal bases.  For the
// isotropic part of the energy the element Hessian is exactly block diagonal in
// this split; the block Hessian used for the direction keeps the 6x6 and 3x3
// diagonal blocks (each made positive semi-definite, then + beta I).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"

namespace emu {

#define DEV __device__ __forceinline__

// value of v in lane `lane` (uniform) for every lane of the wave
DEV double bcast_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The stop flag, read in the same memory round trip as a first value of the
// kernel's own data: the empty asm statement needs both values, so the
// compiler issues the data load before the flag test instead of after it.
template <typename V>
DEV bool stopped(const DevMesh& d, V first) {
  const int done = d.ctl->done;
  __asm__ volatile("" ::"v"(first), "s"(done));
  return done != 0;
}

constexpr double kRs2 = 0.70710678118654752440;  // 1/sqrt(2)

struct DD {
  double hi, lo;
};

DEV void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
DEV DD dd_add(DD x, DD y) {
  double s, e;
  two_sum(x.hi, y.hi, s, e);
  e += x.lo + y.lo;
  double h = s + e;
  return DD{h, e - (h - s)};
}
DEV DD dd_add_d(DD x, double y) {
  double s, e;
  two_sum(x.hi, y, s, e);
  e += x.lo;
  double h = s + e;
  return DD{h, e - (h - s)};
}

// Block-wide reduction of NV double-double values (NT threads, whole waves);
// result valid in thread 0.  Fixed order: a butterfly over the 64 lanes of
// each wave (lane shuffles, no barrier), then thread 0 adds the wave sums in
// wave order after one barrier.
template <int NV, int NT = kBlock>
DEV void block_reduce_dd(DD (&v)[NV], DD* sh) {
  constexpr int W = NT / 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = dd_add(v[k], DD{__shfl_xor(v[k].hi, off), __shfl_xor(v[k].lo, off)});
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * W + wave] = v[k];
  __syncthreads();
  if (t == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      DD a = sh[k * W];
#pragma unroll
      for (int w = 1; w < W; ++w) a = dd_add(a, sh[k * W + w]);
      v[k] = a;
    }
}
// block_reduce_dd of NV double-doubles together with two integer sums, all
// behind one barrier (results in thread 0).
template <int NV, int NT = kBlock>
DEV void block_reduce_dd_int2(DD (&v)[NV], int& a, int& b, DD* sh, int* shi) {
  constexpr int W = NT / 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = dd_add(v[k], DD{__shfl_xor(v[k].hi, off), __shfl_xor(v[k].lo, off)});
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * W + wave] = v[k];
    shi[wave] = a;
    shi[W + wave] = b;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      DD x = sh[k * W];
#pragma unroll
      for (int w = 1; w < W; ++w) x = dd_add(x, sh[k * W + w]);
      v[k] = x;
    }
    a = 0;
    b = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      a += shi[w];
      b += shi[W + w];
    }
  }
}
// Block-wide integer sum (exact, so any order), valid in thread 0.
template <int NT = kBlock>
DEV int block_sum_int(int v, int* sh) {
  constexpr int W = NT / 64;
  const int t = threadIdx.x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  int a = 0;
  if (t == 0)
#pragma unroll
    for (int w = 0; w < W; ++w) a += sh[w];
  return a;
}

// ------------------------------------------------------------------ 3x3 helpers
DEV double det3(const double* a) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}
template <typename T>
DEV void cof3(const T* a, T* c) {
  c[0] = a[4] * a[8] - a[5] * a[7];
  c[1] = a[5] * a[6] - a[3] * a[8];
  c[2] = a[3] * a[7] - a[4] * a[6];
  c[3] = a[2] * a[7] - a[1] * a[8];
  c[4] = a[0] * a[8] - a[2] * a[6];
  c[5] = a[1] * a[6] - a[0] * a[7];
  c[6] = a[1] * a[5] - a[2] * a[4];
  c[7] = a[2] * a[3] - a[0] * a[5];
  c[8] = a[0] * a[4] - a[1] * a[3];
}
// 3x3 (row-major) -> coordinates in the (sym 6, skew 3) orthonormal basis
template <typename T, typename U>
DEV void to_y(const U* X, T* y) {
  y[0] = (T)X[0];
  y[1] = (T)X[4];
  y[2] = (T)X[8];
  y[3] = (T)((X[1] + X[3]) * kRs2);
  y[4] = (T)((X[2] + X[6]) * kRs2);
  y[5] = (T)((X[5] + X[7]) * kRs2);
  y[6] = (T)((X[1] - X[3]) * kRs2);
  y[7] = (T)((X[2] - X[6]) * kRs2);
  y[8] = (T)((X[5] - X[7]) * kRs2);
}
template <typename U>
DEV void from_y(const U* y, double* D) {
  D[0] = y[0];
  D[4] = y[1];
  D[8] = y[2];
  D[1] = (y[3] + y[6]) * kRs2;
  D[3] = (y[3] - y[6]) * kRs2;
  D[2] = (y[4] + y[7]) * kRs2;
  D[6] = (y[4] - y[7]) * kRs2;
  D[5] = (y[5] + y[8]) * kRs2;
  D[7] = (y[5] - y[8]) * kRs2;
}
DEV void s_from6(const double* s, double* S) {
  S[0] = s[0];
  S[4] = s[1];
  S[8] = s[2];
  S[1] = S[3] = s[3] * kRs2;
  S[2] = S[6] = s[4] * kRs2;
  S[5] = S[7] = s[5] * kRs2;
}
DEV void matmul3(const double* A, const double* B, double* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
DEV void matTmul3(const double* A, const double* B, double* C) {  // A^T B
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}

DEV double rsq(double x) { return rsqrt(x); }
DEV float rsq(float x) { return rsqrtf(x); }

// Symmetric eigen-decomposition by cyclic Jacobi, A (N x N, full) overwritten
// with a diagonal, V columns = eigenvectors.
template <typename T, int N>
DEV void jacobi_sym(T (&A)[N][N], T (&V)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) V[i][j] = i == j ? T(1) : T(0);
  for (int sweep = 0; sweep < 16; ++sweep) {
    T off = 0, dia = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      dia += A[i][i] * A[i][i];
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += A[i][j] * A[i][j];
    }
    if (!(off > T(1e-32) * dia)) break;
#pragma unroll
    for (int pp = 0; pp < N; ++pp)
#pragma unroll
      for (int qq = pp + 1; qq < N; ++qq) {
        T apq = A[pp][qq];
        if (apq != T(0)) {
          // tan of the rotation angle, t = sgn(theta) / (|theta| + sqrt(theta^2 + 1))
          // with theta = dqp / (2 apq), written with a single division
          const T dqp = A[qq][qq] - A[pp][pp];
          T t = (dqp >= T(0) ? T(2) : T(-2)) * apq / (fabs(dqp) + sqrt(dqp * dqp + T(4) * apq * apq));
          T c = rsq(t * t + T(1)), s = t * c;
#pragma unroll
          for (int k = 0; k < N; ++k) {
            T akp = A[k][pp], akq = A[k][qq];
            A[k][pp] = c * akp - s * akq;
            A[k][qq] = s * akp + c * akq;
          }
#pragma unroll
          for (int k = 0; k < N; ++k) {
            T apk = A[pp][k], aqk = A[qq][k];
            A[pp][k] = c * apk - s * aqk;
            A[qq][k] = s * apk + c * aqk;
          }
#pragma unroll
          for (int k = 0; k < N; ++k) {
            T vkp = V[k][pp], vkq = V[k][qq];
            V[k][pp] = c * vkp - s * vkq;
            V[k][qq] = s * vkp + c * vkq;
          }
        }
      }
  }
}

// Rotation factor of X: the R in SO(3) maximizing tr(R^T X) (X = U Sig V^T,
// R = U diag(1,1,det(U V^T)) V^T), from the eigenvectors of X^T X: u1, u2 from
// the two largest singular directions, u3 = u1 x u2, v3 = v1 x v2.
DEV void polar3(const double* X, double* R) {
  double M[3][3], V[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i][j] = X[i] * X[j] + X[3 + i] * X[3 + j] + X[6 + i] * X[6 + j];
  jacobi_sym<double, 3>(M, V);
  // order eigenvalues descending
  double la[3] = {M[0][0], M[1][1], M[2][2]};
  int idx[3] = {0, 1, 2};
  if (la[idx[1]] > la[idx[0]]) { int t = idx[0]; idx[0] = idx[1]; idx[1] = t; }
  if (la[idx[2]] > la[idx[1]]) { int t = idx[1]; idx[1] = idx[2]; idx[2] = t; }
  if (la[idx[1]] > la[idx[0]]) { int t = idx[0]; idx[0] = idx[1]; idx[1] = t; }
  double v1[3] = {V[0][idx[0]], V[1][idx[0]], V[2][idx[0]]};
  double v2[3] = {V[0][idx[1]], V[1][idx[1]], V[2][idx[1]]};
  double u1[3], u2[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u1[i] = X[3 * i] * v1[0] + X[3 * i + 1] * v1[1] + X[3 * i + 2] * v1[2];
    u2[i] = X[3 * i] * v2[0] + X[3 * i + 1] * v2[1] + X[3 * i + 2] * v2[2];
  }
  double n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  if (!(n1 > 0)) {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
    return;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) u1[i] /= n1;
  double pr = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) u2[i] -= pr * u1[i];
  double n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  if (!(n2 > 1e-300 + 1e-15 * n1)) {
    // rank <= 1: any unit vector orthogonal to u1
    double ax[3] = {0, 0, 0};
    int k = (fabs(u1[0]) <= fabs(u1[1]) && fabs(u1[0]) <= fabs(u1[2])) ? 0 : (fabs(u1[1]) <= fabs(u1[2]) ? 1 : 2);
    ax[k] = 1.0;
    u2[0] = u1[1] * ax[2] - u1[2] * ax[1];
    u2[1] = u1[2] * ax[0] - u1[0] * ax[2];
    u2[2] = u1[0] * ax[1] - u1[1] * ax[0];
    n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) u2[i] /= n2;
  double u3[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2], u1[0] * u2[1] - u1[1] * u2[0]};
  double v3[3] = {v1[1] * v2[2] - v1[2] * v2[1], v1[2] * v2[0] - v1[0] * v2[2], v1[0] * v2[1] - v1[1] * v2[0]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) R[3 * i + j] = u1[i] * v1[j] + u2[i] * v2[j] + u3[i] * v3[j];
}

// The Jacobi-based polar factor out of line (by value, so nothing is forced
// into scratch memory): the element pass uses it only where the Newton
// iteration declines (inverted or nearly singular elements).
struct Mat3 {
  double v[9];
};
DEV Mat3 load_mat3(const double* a) {
  Mat3 m;
#pragma unroll
  for (int k = 0; k < 9; ++k) m.v[k] = a[k];
  return m;
}
__device__ __noinline__ Mat3 polar3_fallback(Mat3 X) {
  Mat3 R;
  polar3(X.v, R.v);
  return R;
}

// One Newton-Schulz step towards the nearest rotation, R <- R + R (I - R^T R)/2:
// the orthogonality error |R^T R - I| goes to about its square.  Applied to
// the accumulated rotation R <- R Rx after every accepted step, so rounding
// does not build up over thousands of iterations: the energy and gradient are
// taken in S as if R were orthogonal, and on stiff elements (mu vol ~ 600 J)
// an error of 1e-13 in R already shifts dE/dF of the state F = R S by ~1e-10.
DEV void reorthonormalize(double* R) {
  double E[9], RE[9];
  matTmul3(R, R, E);
#pragma unroll
  for (int k = 0; k < 9; ++k) E[k] = (k % 4 == 0 ? 1.0 : 0.0) - E[k];
  matmul3(R, E, RE);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] += 0.5 * RE[k];
}

// Orthogonal polar factor by the scaled Newton iteration
//   X <- (z X + X^{-T} / z) / 2,  z = |det X|^{-1/3}  (determinant scaling),
// which converges quadratically to the rotation of X when det X > 0.  The
// scaling is applied while det X is away from 1 (|det X - 1| > 1e-2); the
// unscaled steps near convergence stop once a step changes X by <= 1e-15
// relative.  Returns false (R untouched) for det X <= 0, a tiny determinant or
// no convergence in 12 steps; the caller then uses polar3.
DEV bool polar3_newton(const double* X0, double* R) {
  double X[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = X0[k];
  double nx = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) nx += X[k] * X[k];
  double dt = det3(X);
  if (!(dt > 1e-12 * nx * sqrt(nx))) return false;
  for (int it = 0; it < 12; ++it) {
    double C[9];
    cof3<double>(X, C);  // X^{-T} = cof(X) / det X
    const bool scale = fabs(dt - 1.0) > 1e-2;
    const double z = scale ? cbrt(1.0 / dt) : 1.0;
    const double a = 0.5 * z, b = 0.5 / (z * dt);
    double diff = 0, nrm = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double y = a * X[k] + b * C[k];
      diff += (y - X[k]) * (y - X[k]);
      nrm += y * y;
      X[k] = y;
    }
    if (!scale && diff <= 1e-30 * nrm) {
#pragma unroll
      for (int k = 0; k < 9; ++k) R[k] = X[k];
      return true;
    }
    dt = det3(X);
    if (!(dt > 0)) return false;
  }
  return false;
}

// ------------------------------------------------------------------ element Hessian
// Core 9x9 Hessian of Psi at the symmetric S (row-major index 3a+i for F_ai):
//   mu delta + kappa d2J/dF2 + phi (I (x) u u^T),  kappa = lhat (J-1) - mu,
// with d2J/dF_ai dF_bj = eps_abc eps_ijk S_ck.  (lhat cof cof^T is added to the
// symmetric block separately.)
DEV int eps2(int a, int b) { return (b == (a + 1) % 3) ? 1 : -1; }

template <typename T>
DEV T hcore(int A, int B, const T* S, T mu, T kappa, T phi, const T* u) {
  const int a = A / 3, i = A % 3, b = B / 3, j = B % 3;
  T v = 0;
  if (a == b && i == j) v += mu;
  if (a != b && i != j) v += kappa * T(eps2(a, b) * eps2(i, j)) * S[3 * (3 - a - b) + (3 - i - j)];
  if (a == b) v += phi * u[i] * u[j];
  return v;
}

// basis nonzeros: symmetric l = 0..5, skew m = 0..2 (index 3a+i, value)
__device__ constexpr int kYn[9] = {1, 1, 1, 2, 2, 2, 2, 2, 2};
__device__ constexpr int kYi[9][2] = {{0, 0}, {4, 4}, {8, 8}, {1, 3}, {2, 6}, {5, 7}, {1, 3}, {2, 6}, {5, 7}};
__device__ constexpr double kYv[9][2] = {{1, 0}, {1, 0}, {1, 0}, {kRs2, kRs2}, {kRs2, kRs2}, {kRs2, kRs2},
                                         {kRs2, -kRs2}, {kRs2, -kRs2}, {kRs2, -kRs2}};


// For each matrix entry A = 3a+i: the (up to two) basis elements with a nonzero
// there and the value: diagonal -> symmetric basis only; off-diagonal ->
// symmetric (1/sqrt2) and skew (+1/sqrt2 above, -1/sqrt2 below the diagonal).
__device__ constexpr int kYof[9][2] = {{0, -1}, {3, 6}, {4, 7}, {3, 6}, {1, -1}, {5, 8}, {4, 7}, {5, 8}, {2, -1}};
__device__ constexpr double kYvf[9][2] = {{1, 0}, {kRs2, kRs2}, {kRs2, kRs2}, {kRs2, -kRs2}, {1, 0},
                                          {kRs2, kRs2}, {kRs2, -kRs2}, {kRs2, -kRs2}, {1, 0}};

template <typename T>
DEV T hproj(int y, int z, const T* S, T mu, T kappa, T phi, const T* u) {
  T s = 0;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (p < kYn[y] && q < kYn[z])
        s += T(kYv[y][p]) * T(kYv[z][q]) * hcore<T>(kYi[y][p], kYi[z][q], S, mu, kappa, phi, u);
  return s;
}

// Packed lower Cholesky of a full N x N matrix; false if not positive definite.
// rdiag (optional) receives the reciprocals of the diagonal.
template <typename T, int N>
DEV bool chol_packed(const T (&A)[N][N], T* L, T* rdiag = nullptr) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T s = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j * (j + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
    if (!(s > T(0))) return false;
    const T rd = rsq(s);  // 1 / sqrt(s) without a division
    L[j * (j + 1) / 2 + j] = s * rd;
    if (rdiag) rdiag[j] = rd;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
      L[i * (i + 1) / 2 + j] = t * rd;
    }
  }
  return true;
}
template <typename T, int N>
DEV void chol_solve(const T* L, T* x) {  // in place: L L^T x = b
  T rd[N];
#pragma unroll
  for (int i = 0; i < N; ++i) rd[i] = T(1) / L[i * (i + 1) / 2 + i];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T t = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[i * (i + 1) / 2 + k] * x[k];
    x[i] = t * rd[i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T t = x[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) t -= L[k * (k + 1) / 2 + i] * x[k];
    x[i] = t * rd[i];
  }
}
// P = (L L^T)^{-1} = L^{-T} L^{-1}, packed lower, from the packed lower factor L.
template <typename T, int N>
DEV void chol_inverse(const T* L, T* P) {
  T Li[N * (N + 1) / 2];
#pragma unroll
  for (int c = 0; c < N; ++c) Li[c * (c + 1) / 2 + c] = T(1) / L[c * (c + 1) / 2 + c];
#pragma unroll
  for (int c = 0; c < N; ++c) {
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      T v = 0;
#pragma unroll
      for (int k = c; k < r; ++k) v += L[r * (r + 1) / 2 + k] * Li[k * (k + 1) / 2 + c];
      Li[r * (r + 1) / 2 + c] = -v * Li[r * (r + 1) / 2 + r];
    }
  }
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      T v = 0;
#pragma unroll
      for (int k = r; k < N; ++k) v += Li[k * (k + 1) / 2 + r] * Li[k * (k + 1) / 2 + c];
      P[r * (r + 1) / 2 + c] = v;
    }
}
// The same inverse stored straight to memory (out[(packed index) * m + i]) with
// x <- P x on the way, holding only L^{-1} in registers: x = L^{-T} (L^{-1} x),
// and every entry of P is stored as soon as it is formed.  rdiag: the
// reciprocals of L's diagonal from the factorization.
template <typename T, int N>
DEV void chol_inverse_apply_store(const T* L, const T* rdiag, T* x, T* out, int m, int i) {
  T Li[N * (N + 1) / 2];
#pragma unroll
  for (int c = 0; c < N; ++c) Li[c * (c + 1) / 2 + c] = rdiag[c];
#pragma unroll
  for (int c = 0; c < N; ++c) {
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      T v = 0;
#pragma unroll
      for (int k = c; k < r; ++k) v += L[r * (r + 1) / 2 + k] * Li[k * (k + 1) / 2 + c];
      Li[r * (r + 1) / 2 + c] = -v * Li[r * (r + 1) / 2 + r];
    }
  }
  T z[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    T v = 0;
#pragma unroll
    for (int k = 0; k <= r; ++k) v += Li[r * (r + 1) / 2 + k] * x[k];
    z[r] = v;
  }
#pragma unroll
  for (int c = 0; c < N; ++c) {
    T v = 0;
#pragma unroll
    for (int r = c; r < N; ++r) v += Li[r * (r + 1) / 2 + c] * z[r];
    x[c] = v;
  }
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      T v = 0;
#pragma unroll
      for (int k = r; k < N; ++k) v += Li[k * (k + 1) / 2 + r] * Li[k * (k + 1) / 2 + c];
      out[(int64_t)(r * (r + 1) / 2 + c) * m + i] = v;
    }
}
// x <- P x for a packed (lower) symmetric P.
template <typename T, int N>
DEV void sym_apply(const T* P, T* x) {
  T y[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    T v = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) v += P[r >= c ? r * (r + 1) / 2 + c : c * (c + 1) / 2 + r] * x[c];
    y[r] = v;
  }
#pragma unroll
  for (int r = 0; r < N; ++r) x[r] = y[r];
}

// A <- its positive semi-definite part (eigenvalues < 0 -> 0), by Jacobi.
template <typename T, int N>
DEV void clamp_psd_jacobi(T (&A)[N][N]) {
  T V[N][N];
  jacobi_sym<T, N>(A, V);
  T lam[N];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = A[k][k] > T(0) ? A[k][k] : T(0);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T s = 0;
#pragma unroll
      for (int k = 0; k < N; ++k) s += V[i][k] * lam[k] * V[j][k];
      A[i][j] = s;
    }
}

// The same projection for the rare indefinite 6x6 block, in place on a full
// symmetric matrix W in LDS with the eigenvectors in V (LDS), rolled loops:
// no scratch memory and few registers, so that it does not set the register
// allocation of the Hessian pass.
template <typename T, int N>
DEV void clamp_psd_jacobi_lds(T (*W)[N], T (*V)[N]) {
#pragma unroll 1
  for (int i = 0; i < N; ++i)
#pragma unroll 1
    for (int j = 0; j < N; ++j) V[i][j] = i == j ? T(1) : T(0);
#pragma unroll 1
  for (int sweep = 0; sweep < 16; ++sweep) {
    T off = 0, dia = 0;
#pragma unroll 1
    for (int i = 0; i < N; ++i) {
      dia += W[i][i] * W[i][i];
#pragma unroll 1
      for (int j = i + 1; j < N; ++j) off += W[i][j] * W[i][j];
    }
    if (!(off > T(1e-32) * dia)) break;
#pragma unroll 1
    for (int pp = 0; pp < N; ++pp)
#pragma unroll 1
      for (int qq = pp + 1; qq < N; ++qq) {
        const T apq = W[pp][qq];
        if (apq != T(0)) {
          const T dqp = W[qq][qq] - W[pp][pp];
          const T t = (dqp >= T(0) ? T(2) : T(-2)) * apq / (fabs(dqp) + sqrt(dqp * dqp + T(4) * apq * apq));
          const T c = rsq(t * t + T(1)), s = t * c;
#pragma unroll 1
          for (int k = 0; k < N; ++k) {
            const T akp = W[k][pp], akq = W[k][qq];
            W[k][pp] = c * akp - s * akq;
            W[k][qq] = s * akp + c * akq;
          }
#pragma unroll 1
          for (int k = 0; k < N; ++k) {
            const T apk = W[pp][k], aqk = W[qq][k];
            W[pp][k] = c * apk - s * aqk;
            W[qq][k] = s * apk + c * aqk;
          }
#pragma unroll 1
          for (int k = 0; k < N; ++k) {
            const T vkp = V[k][pp], vkq = V[k][qq];
            V[k][pp] = c * vkp - s * vkq;
            V[k][qq] = s * vkp + c * vkq;
          }
        }
      }
  }
  T lam[N];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = W[k][k] > T(0) ? W[k][k] : T(0);
#pragma unroll 1
  for (int i = 0; i < N; ++i)
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
      T sm = 0;
#pragma unroll
      for (int k = 0; k < N; ++k) sm += V[i][k] * lam[k] * V[j][k];
      W[i][j] = sm;
    }
}

// cos(acos(r) / 3) for r in [-1, 1]: the root c in [1/2, 1] of
// 4 c^3 - 3 c = r (cos 3t = 4 cos^3 t - 3 cos t).  With c = 1/2 + u this is
// 6 u^2 + 4 u^3 = 1 + r, a simple root u >= 0 for every r > -1 (at r = -1
// the cubic in c has a double root, so Newton on c would stall there).
// Double precision: a single-precision start (u ~ sqrt((1 + r) / 6) when
// 1 + r is small), then three Newton steps; as accurate as acos and cos in
// double (checked against a symmetric eigensolver on random and nearly
// degenerate 3x3 matrices), without their cost.
DEV float cos_third_acos(float r) { return cosf(acosf(r) * (1.0f / 3.0f)); }
DEV double cos_third_acos(double r) {
  const double t = 1.0 + r;
  double u = (double)cosf(acosf((float)r) * (1.0f / 3.0f)) - 0.5;
  if (t < 1e-2) u = sqrt(t * (1.0 / 6.0));
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    const double dg = 12.0 * u * (1.0 + u);
    if (dg > 0.0) u -= ((6.0 + 4.0 * u) * u * u - t) / dg;
  }
  return 0.5 + u;
}

// Unit eigenvector of the symmetric 3x3 A for its simple eigenvalue lam: the
// longest of the cross products of two rows of A - lam I, normalized.
template <typename T>
DEV void eigvec3(const T (&A)[3][3], T lam, T* v) {
  const T r[3][3] = {{A[0][0] - lam, A[0][1], A[0][2]},
                     {A[1][0], A[1][1] - lam, A[1][2]},
                     {A[2][0], A[2][1], A[2][2] - lam}};
  T c[3][3];
  const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  T best = -1;
  int kb = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T* a = r[pr[k][0]];
    const T* b = r[pr[k][1]];
    c[k][0] = a[1] * b[2] - a[2] * b[1];
    c[k][1] = a[2] * b[0] - a[0] * b[2];
    c[k][2] = a[0] * b[1] - a[1] * b[0];
    const T n = c[k][0] * c[k][0] + c[k][1] * c[k][1] + c[k][2] * c[k][2];
    if (n > best) {
      best = n;
      kb = k;
    }
  }
  const T s = rsq(best);
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = (kb == 0 ? c[0][i] : (kb == 1 ? c[1][i] : c[2][i])) * s;
}

// PSD part of a symmetric 3x3 in closed form: the eigenvalues from the
// trigonometric solution of the characteristic cubic (shifted by the mean
// eigenvalue and scaled), then A+ = A - e3 v3 v3^T (one negative eigenvalue)
// or e1 v1 v1^T (two).  Returns false, leaving A unchanged, when the kept and
// the dropped eigenvalues are closer than 1e-4 of the largest magnitude (the
// eigenvector would be inaccurate); the caller then uses Jacobi.
template <typename T>
DEV bool clamp_psd3_closed(T (&A)[3][3]) {
  const T q = (A[0][0] + A[1][1] + A[2][2]) * T(1.0 / 3.0);
  const T b00 = A[0][0] - q, b11 = A[1][1] - q, b22 = A[2][2] - q;
  const T a01 = A[0][1], a02 = A[0][2], a12 = A[1][2];
  const T p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const T p = sqrt((b00 * b00 + b11 * b11 + b22 * b22 + T(2) * p1) * T(1.0 / 6.0));
  if (!(p > T(0))) {  // A = q I
    if (q < T(0))
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[i][j] = T(0);
    return true;
  }
  const T ip = T(1) / p;
  const T c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip, c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
  T r = T(0.5) * (c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02));
  r = r < T(-1) ? T(-1) : (r > T(1) ? T(1) : r);
  // eigenvalues q + 2 p cos(phi + 2 pi k / 3), phi = acos(r) / 3
  const T c = cos_third_acos(r);
  const T sn = sqrt(c < T(1) ? T(1) - c * c : T(0));  // sin(phi), phi in [0, pi/3]
  const T e1 = q + T(2) * p * c;
  const T e3 = q - p * (c + T(1.7320508075688772935) * sn);  // 2 p cos(phi + 2 pi / 3)
  const T e2 = T(3) * q - e1 - e3;
  const T scale = fabs(e1) > fabs(e3) ? fabs(e1) : fabs(e3);
  if (!(e1 > T(0))) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) A[i][j] = T(0);
    return true;
  }
  if (!(e3 < T(0))) return true;  // already semi-definite
  T v[3];
  if (e2 >= T(0)) {
    if (!(e2 - e3 > T(1e-4) * scale)) return false;
    eigvec3<T>(A, e3, v);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) A[i][j] -= e3 * v[i] * v[j];
  } else {
    if (!(e1 - e2 > T(1e-4) * scale)) return false;
    eigvec3<T>(A, e1, v);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) A[i][j] = e1 * v[i] * v[j];
  }
  return true;
}

// Make A positive semi-definite (eigenvalues < 0 -> 0) unless a Cholesky
// factorization already succeeds; then add beta I and factor.  Returns 1 if
// the clamp changed A.  3x3 blocks take the closed form where it is accurate.
// L = chol(A + beta I) for a positive semi-definite A (A is modified).
template <typename T, int N>
DEV void add_factor(T (&A)[N][N], T beta, T* L, T* rdiag = nullptr) {
#pragma unroll
  for (int k = 0; k < N; ++k) A[k][k] += beta;
  if (!chol_packed<T, N>(A, L, rdiag)) {
    // beta > 0 makes this positive definite; guard against beta == 0 with a tiny shift
    T sc = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) sc = A[k][k] > sc ? A[k][k] : sc;
#pragma unroll
    for (int k = 0; k < N; ++k) A[k][k] += T(1e-12) * sc + T(1e-300);
    chol_packed<T, N>(A, L, rdiag);
  }
}

template <typename T, int N>
DEV int clamp_add_factor(T (&A)[N][N], T beta, T* L, T* rdiag = nullptr) {
  int clamped = 0;
  if (!chol_packed<T, N>(A, L)) {
    if constexpr (N == 3) {
      if (!clamp_psd3_closed<T>(A)) clamp_psd_jacobi<T, 3>(A);
    } else {
      clamp_psd_jacobi<T, N>(A);
    }
    clamped = 1;
  }
  add_factor<T, N>(A, beta, L, rdiag);
  return clamped;
}

// Coupled 9x9 blocks (the mesh option hessian_blocks = 1).  In the rotated
// frame dF = R dX the isotropic part of the element Hessian is block diagonal
// (6x6 symmetric, 3x3 skew); it is clamped and factored per block exactly as in
// the split form (D).  The fiber term a k_f |F u|^2 = a k_f |X u|^2 is a convex
// quadratic whose Hessian 2 a k_f vol (I (x) u u^T) is positive semi-definite
// of rank 3: V V^T, with column c of V the y-coordinates of sqrt(2 a k_f vol)
// e_c u^T.  The block H = D + V V^T keeps the fiber's coupling of the
// symmetric and skew parts, and
//   H^{-1} = D^{-1} - D^{-1} V K^{-1} V^T D^{-1},  K = I + V^T D^{-1} V (3x3),
// so only K^{-1} (6 values) is stored after D^{-1}'s 27.
constexpr int kLfSplit = 27;
constexpr int kLfCoupled = 33;

template <typename T>
DEV void fiber_cols(const T* u, T s, T (&V)[9][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T M[9], y[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) M[k] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * c + j] = s * u[j];
    to_y<T, T>(M, y);
#pragma unroll
    for (int k = 0; k < 9; ++k) V[k][c] = y[k];
  }
}
// sqrt(2 a k_f vol) of element i (0 for passive tets or zero activation).
DEV double fiber_scale(const DevMesh& d, int i) {
  const int g = d.grp[i];
  const double a = g >= 0 ? d.act[g] : 0.0;
  return a > 0.0 ? sqrt(2.0 * a * d.kf * d.vol[i]) : 0.0;
}
template <typename T>
DEV void fiber_V(const DevMesh& d, int i, T (&V)[9][3]) {
  const int m = d.m;
  const T u[3] = {(T)d.fib[i], (T)d.fib[m + i], (T)d.fib[2 * m + i]};
  fiber_cols<T>(u, (T)fiber_scale(d, i), V);
}
// x <- D^{-1} x with the stored split inverses (6x6 and 3x3, packed)
template <typename T>
DEV void split_apply(const T* Ds, const T* Dk, T* x) {
  sym_apply<T, 6>(Ds, x);
  sym_apply<T, 3>(Dk, x + 6);
}
// x <- H^{-1} x: the split inverses, then (coupled form) the rank-3 correction
template <typename T, bool kC>
DEV void hinv_apply(const DevMesh& d, int i, const T* Ds, const T* Dk, T* x) {
  if constexpr (kC) {
    const T* Lf = (const T*)d.Lf;
    const int m = d.m;
    T V[9][3], Ki[6];
    fiber_V<T>(d, i, V);
#pragma unroll
    for (int k = 0; k < 6; ++k) Ki[k] = Lf[(kLfSplit + k) * m + i];
    split_apply<T>(Ds, Dk, x);
    T t[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T v = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) v += V[k][c] * x[k];
      t[c] = v;
    }
    sym_apply<T, 3>(Ki, t);
    T w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = V[k][0] * t[0] + V[k][1] * t[1] + V[k][2] * t[2];
    split_apply<T>(Ds, Dk, w);
#pragma unroll
    for (int k = 0; k < 9; ++k) x[k] -= w[k];
  } else {
    split_apply<T>(Ds, Dk, x);
  }
}
// Coupled form, after the split inverses of element i are stored and gbar
// holds D^{-1} g: form and store K^{-1}, and finish gbar = H^{-1} g.
template <typename T>
DEV void coupled_finish(const DevMesh& d, int i) {
  const int m = d.m;
  T* Lf = (T*)d.Lf;
  T* gbar = (T*)d.gbar;
  T Ki[6] = {T(1), T(0), T(1), T(0), T(0), T(1)};
  if (fiber_scale(d, i) > 0.0) {
    T Ds[21], Dk[6], V[9][3], W[9][3];
#pragma unroll
    for (int k = 0; k < 21; ++k) Ds[k] = Lf[k * m + i];
#pragma unroll
    for (int k = 0; k < 6; ++k) Dk[k] = Lf[(21 + k) * m + i];
    fiber_V<T>(d, i, V);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T col[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) col[k] = V[k][c];
      split_apply<T>(Ds, Dk, col);
#pragma unroll
      for (int k = 0; k < 9; ++k) W[k][c] = col[k];
    }
    T K[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        T v = a == b ? T(1) : T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) v += V[k][a] * W[k][b];
        K[a][b] = v;
      }
    K[0][1] = K[1][0] = T(0.5) * (K[0][1] + K[1][0]);
    K[0][2] = K[2][0] = T(0.5) * (K[0][2] + K[2][0]);
    K[1][2] = K[2][1] = T(0.5) * (K[1][2] + K[2][1]);
    T Kf[6];
    chol_packed<T, 3>(K, Kf);  // K >= I: positive definite
    chol_inverse<T, 3>(Kf, Ki);
    T g[9], t[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) g[k] = gbar[k * m + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T v = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) v += V[k][c] * g[k];
      t[c] = v;
    }
    sym_apply<T, 3>(Ki, t);
#pragma unroll
    for (int k = 0; k < 9; ++k) gbar[k * m + i] = g[k] - (W[k][0] * t[0] + W[k][1] * t[1] + W[k][2] * t[2]);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) Lf[(kLfSplit + k) * m + i] = Ki[k];
}

// ------------------------------------------------------------------ element data access
struct Elem {
  int32_t v[4];
  double b[4][3];
  double vol, mu, lhat, w, u[3], a;
};

DEV void load_elem(const DevMesh& d, int i, Elem& e) {
  const int m = d.m;
#pragma unroll
  for (int k = 0; k < 4; ++k) e.v[k] = d.vid[k * m + i];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) e.b[k][c] = d.dminv[(3 * k + c) * m + i];
#pragma unroll
  for (int c = 0; c < 3; ++c) e.b[3][c] = -(e.b[0][c] + e.b[1][c] + e.b[2][c]);
  e.vol = d.vol[i];
  e.mu = d.mu[i];
  e.lhat = d.lhat[i];
  e.w = d.w[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) e.u[c] = d.fib[c * m + i];
  int g = d.grp[i];
  e.a = g >= 0 ? d.act[g] : 0.0;
}

// A[c][dd] = sum_v x[v][c] b_v[dd]  (compatible gradient of a vertex field)
DEV void gather_grad(const double* x, const Elem& e, double* A) {
  double xv[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[k][c] = x[3 * e.v[k] + c];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int dd = 0; dd < 3; ++dd)
      A[3 * c + dd] = xv[0][c] * e.b[0][dd] + xv[1][c] * e.b[1][dd] + xv[2][c] * e.b[2][dd] + xv[3][c] * e.b[3][dd];
}

// ACAP right-hand side contributions of the field F: w b_v . F[c,:]
DEV void write_contrib(const DevMesh& d, int i, const Elem& e, const double* F) {
  double* o = d.contrib + (int64_t)12 * i;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      o[3 * k + c] = e.w * (F[3 * c] * e.b[k][0] + F[3 * c + 1] * e.b[k][1] + F[3 * c + 2] * e.b[k][2]);
}

DEV void load_R(const DevMesh& d, int i, double* R) {
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = d.R[k * d.m + i];
}
DEV void load_S(const DevMesh& d, int i, double* S) {
  double s[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = d.S[k * d.m + i];
  s_from6(s, S);
}

// ------------------------------------------------------------------ kernels
__global__ void __launch_bounds__(kBlock) k_init_rest(DevMesh d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
#pragma unroll
  for (int k = 0; k < 9; ++k) d.R[k * d.m + i] = (k % 4 == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) d.S[k * d.m + i] = k < 3 ? 1.0 : 0.0;
}

// F (internal element order, [m][9]) -> R, S
__global__ void __launch_bounds__(kBlock) k_set_F(DevMesh d, const double* F, const int32_t* eold) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  const double* f = F + (int64_t)9 * eold[i];
  double X[9], R[9], S[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = f[k];
  polar3(X, R);
  matTmul3(R, X, S);
  double y[9];
  to_y<double, double>(S, y);
#pragma unroll
  for (int k = 0; k < 9; ++k) d.R[k * d.m + i] = R[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) d.S[k * d.m + i] = y[k];
}

// F = R S -> user order [m][9]
__global__ void __launch_bounds__(kBlock) k_get_F(DevMesh d, double* F, const int32_t* eold) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  double R[9], S[9], X[9];
  load_R(d, i, R);
  load_S(d, i, S);
  matmul3(R, S, X);
  double* f = F + (int64_t)9 * eold[i];
#pragma unroll
  for (int k = 0; k < 9; ++k) f[k] = X[k];
}

// direction d = -p in F coordinates, user order [m][9]
__global__ void __launch_bounds__(kBlock) k_get_dir(DevMesh d, double* out, const int32_t* eold) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  double R[9], y[9], D[9], X[9];
  load_R(d, i, R);
#pragma unroll
  for (int k = 0; k < 9; ++k) y[k] = -d.p[k * d.m + i];
  from_y<double>(y, D);
  matmul3(R, D, X);
  double* f = out + (int64_t)9 * eold[i];
#pragma unroll
  for (int k = 0; k < 9; ++k) f[k] = X[k];
}

// contributions of F = R S (fresh ACAP solve)
__global__ void __launch_bounds__(kBlock) k_scatter_F(DevMesh d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  Elem e;
  load_elem(d, i, e);
  double R[9], S[9], F[9];
  load_R(d, i, R);
  load_S(d, i, S);
  matmul3(R, S, F);
  write_contrib(d, i, e, F);
}

// right-hand side of the ACAP solve: fixed-order sum of element contributions
// at each free vertex, plus (optionally) the constant pinned term -L_fp qbar_p
// kRhsLanes lanes per vertex take interleaved entries of its incidence list and
// are added in a fixed order.
constexpr int kRhsLanes = 8;
// Workgroups are dispatched to the 8 XCDs in turn (workgroup b to XCD b % 8),
// and each XCD has its own L2.  Passes whose neighbouring workgroups share
// data (elements sharing vertices, vertices sharing elements) renumber the
// workgroups so that each XCD gets a contiguous range: XCD x takes logical
// blocks [x q + min(x, r), ...) for nb = 8 q + r.  A bijection on [0, nb).
DEV int xcd_block(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}

DEV void b_rhs(const DevMesh& d, int bid, int add_pin, int check_done) {
  const int lb = xcd_block(bid, (d.nf * kRhsLanes + kBlock - 1) / kBlock);
  const int f = lb * (kBlock / kRhsLanes) + (int)threadIdx.x / kRhsLanes;
  if (check_done && stopped(d, f < d.nf ? d.inc_ptr[f] : 0)) return;
  const int sub = threadIdx.x % kRhsLanes;
  double acc[3] = {0, 0, 0};
  if (f < d.nf) {
    const int k0 = d.inc_ptr[f], k1 = d.inc_ptr[f + 1];
    // unrolled so that several incidence codes, then their contributions,
    // are in flight together (two dependent loads per entry)
#pragma unroll 4
    for (int k = k0 + sub; k < k1; k += kRhsLanes) {
      const int code = d.inc[k];
      const double* src = d.contrib + (int64_t)12 * (code >> 2) + 3 * (code & 3);
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += src[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int off = 1; off < kRhsLanes; off <<= 1) acc[c] += __shfl_xor(acc[c], off);
  if (f >= d.nf || sub != 0) return;
  if (add_pin)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += d.pin_rhs[3 * f + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) d.rhs[3 * f + c] = acc[c];
}
__global__ void __launch_bounds__(kBlock) k_rhs(DevMesh d, int add_pin, int check_done) { b_rhs(d, blockIdx.x, add_pin, check_done); }

// Packed-row products of the triangular sweeps.  A workgroup (4 waves) owns
// 256 / LPR output rows; each wave splits into 64 / LPR groups of LPR lanes and
// a group computes one row: lanes stride the packed row (LPR consecutive
// doubles per step, 4 steps in flight), then reduce within the group.  Work
// items of supernodes with long rows on sparse levels use LPR = 32 (8 rows per
// workgroup) so that the few supernodes near the root still spread over many
// compute units; the rest use LPR = 8 (32 rows).  The vector the rows multiply
// lives in LDS, loaded in chunks of kVecChunk.
constexpr int kVecChunk = 1536;  // 36 KB of LDS: four workgroups per CU, and the merged root (<= 1536 wide) in one chunk
// Levels whose supernodes are all narrow (no 32-lane rows, vectors of a few
// hundred entries) run a variant with a 12 KB chunk and at most 64 VGPRs:
// eight workgroups per CU instead of four, for levels whose short items are
// bound by the latency of the frontal gather, not by bytes.
constexpr int kVecChunkNarrow = kNarrowChunk;

template <bool kFwd, int LPR>
DEV void row_products(const double* __restrict__ V, int64_t base, int w, int h, int r0, int nrows,
                      const double* vec, int vbase, int vlen, double (&acc)[3]) {
  constexpr int G = 64 / LPR;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane / LPR, l = lane % LPR;
  const int rr = wave * G + g;  // row handled by this group
  const int r = r0 + rr;
  double a0 = 0, a1 = 0, a2 = 0;
  if (rr < nrows) {
    // forward: row r has length (r < w ? r+1 : w), starts at column 0
    // backward: row r (a column of L) covers vector entries [r, h)
    int64_t roff;
    int lo, hi;
    if (kFwd) {
      roff = r < w ? (int64_t)r * (r + 1) / 2 : (int64_t)w * (w + 1) / 2 + (int64_t)(r - w) * w;
      lo = 0;
      hi = r < w ? r + 1 : w;
    } else {
      roff = (int64_t)r * h - (int64_t)r * (r - 1) / 2;
      lo = r;
      hi = h;
    }
    // intersect with the vector chunk [vbase, vbase + vlen)
    const int c0 = max(lo, vbase), c1 = min(hi, vbase + vlen);
    const double* row = V + base + roff - lo;
    int c = c0 + l;
    for (; c + 7 * LPR < c1; c += 8 * LPR) {  // 8 loads in flight per lane
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = row[c + u * LPR];
      const double* v0 = vec + 3 * (c - vbase);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a0 += x[u] * v0[3 * u * LPR];
        a1 += x[u] * v0[3 * u * LPR + 1];
        a2 += x[u] * v0[3 * u * LPR + 2];
      }
    }
    for (; c + 3 * LPR < c1; c += 4 * LPR) {
      const double x0 = row[c], x1 = row[c + LPR], x2 = row[c + 2 * LPR], x3 = row[c + 3 * LPR];
      const double* v0 = vec + 3 * (c - vbase);
      a0 += x0 * v0[0] + x1 * v0[3 * LPR] + x2 * v0[6 * LPR] + x3 * v0[9 * LPR];
      a1 += x0 * v0[1] + x1 * v0[3 * LPR + 1] + x2 * v0[6 * LPR + 1] + x3 * v0[9 * LPR + 1];
      a2 += x0 * v0[2] + x1 * v0[3 * LPR + 2] + x2 * v0[6 * LPR + 2] + x3 * v0[9 * LPR + 2];
    }
    for (; c < c1; c += LPR) {
      const double x0 = row[c];
      const double* v0 = vec + 3 * (c - vbase);
      a0 += x0 * v0[0];
      a1 += x0 * v0[1];
      a2 += x0 * v0[2];
    }
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off);
    a1 += __shfl_xor(a1, off);
    a2 += __shfl_xor(a2, off);
  }
  acc[0] += a0;
  acc[1] += a1;
  acc[2] += a2;
}

// Work items carry the lanes-per-row choice in bit 30 of their first row.
constexpr int kItemWide = kItemWideBit;

// Forward sweep of one level.  Work item (s, r0): rows [r0, r0 + 256/LPR) of
// supernode s.  Frontal vector f = [rhs at the columns; 0] + children's update
// vectors; rows r < w give y = Linv f_top, rows r >= w give u = f_r - M_r f_top,
// written to the slot row of the parent front position that row r lands on.
// Sum of the children's slot rows of front position pos (zero where a child
// has no update row), added in child order.
DEV void gather_updates(const DevMesh& d, const SweepItem& it, int pos, double& a0, double& a1, double& a2) {
  const double* u = d.slots + 3 * ((int64_t)it.slotbase + pos);
  const int64_t step = 3 * (int64_t)it.h;
  int k = 0;
  for (; k + 1 < it.nslot; k += 2, u += 2 * step) {
    const double x0 = u[0], x1 = u[1], x2 = u[2];
    const double y0 = u[step], y1 = u[step + 1], y2 = u[step + 2];
    a0 += x0;
    a1 += x1;
    a2 += x2;
    a0 += y0;
    a1 += y1;
    a2 += y2;
  }
  if (k < it.nslot) {
    a0 += u[0];
    a1 += u[1];
    a2 += u[2];
  }
}

template <int LPR, int CH>
DEV void fwd_item(const DevMesh& d, const SweepItem& it, int r0, double* ft) {
  const int w = it.w, h = it.h, col0 = it.col0;
  const int t = threadIdx.x;
  const int nrows = min(256 / LPR, h - r0);
  // the rows of this item need f_top entries [0, min(w, r0 + nrows))
  const int need = min(w, r0 + nrows);
  double acc[3] = {0, 0, 0};
  // children's updates to this group's row (rows below the diagonal block),
  // requested first so they overlap the frontal assembly
  const int lane = t & 63, wave = t >> 6, g = lane / LPR, l = lane % LPR;
  const int rr = wave * (64 / LPR) + g;
  const int r = r0 + rr;
  double b0 = 0, b1 = 0, b2 = 0;
  int32_t orow = 0;
  if (l == 0 && rr < nrows && r >= w) {
    orow = d.dst[it.rowoff + r - w];
    gather_updates(d, it, r, b0, b1, b2);
  }
  for (int vb = 0; vb < need; vb += CH) {
    const int vl = min(CH, need - vb);
    __syncthreads();
    for (int k = t; k < vl; k += kBlock) {
      const int c = vb + k;
      double a0 = d.rhs[3 * (col0 + c)], a1 = d.rhs[3 * (col0 + c) + 1], a2 = d.rhs[3 * (col0 + c) + 2];
      gather_updates(d, it, c, a0, a1, a2);
      ft[3 * k] = a0;
      ft[3 * k + 1] = a1;
      ft[3 * k + 2] = a2;
    }
    __syncthreads();
    row_products<true, LPR>(d.vals, it.valoff, w, h, r0, nrows, ft, vb, vl, acc);
  }
  if (l == 0 && rr < nrows) {
    if (r < w) {
      d.ybuf[3 * (col0 + r)] = acc[0];
      d.ybuf[3 * (col0 + r) + 1] = acc[1];
      d.ybuf[3 * (col0 + r) + 2] = acc[2];
    } else {
      double* o = d.slots + 3 * (int64_t)orow;
      o[0] = b0 - acc[0];
      o[1] = b1 - acc[1];
      o[2] = b2 - acc[2];
    }
  }
}
// Column form (levels of narrow supernodes, w <= kColW): one wave per item of
// kColRows rows; lane l computes row r = r0 + l from the column-major copy of
// the block (tvals: column c holds rows c .. h-1), so every column step is one
// coalesced load across the wave, while the frontal vector, gathered once per
// item into the wave's LDS slice ft, is read as a broadcast.  The block
// entries stream in chunks of kColChunk columns, two chunks in flight: the
// first chunk and the children's updates of the lane's output row are
// requested before the frontal gather.
constexpr int kColChunk = 8;
// columns cb .. cb + kColChunk - 1 of row rr (zero past the lane's nc).  blk
// is the supernode's column-major block, column c starting at
// c h - c (c - 1) / 2 with entry r at index r - c; every load is at a column
// clamped to w - 1 and a row clamped to h - 1 by the caller, so it stays
// inside the block, and the column base is the same for the whole wave.
DEV void col_chunk(const double* blk, int h, int w, int rr, int nc, int cb, double (&x)[kColChunk]) {
#pragma unroll
  for (int u = 0; u < kColChunk; ++u) {
    const int c = min(cb + u, w - 1);
    const double* cp = blk + ((int64_t)c * h - (int64_t)c * (c - 1) / 2 - c);
    const double v = cp[rr];
    x[u] = cb + u < nc ? v : 0.0;
  }
}
DEV void col_fma(const double (&x)[kColChunk], const double* ft, int cb, double& a0, double& a1, double& a2) {
#pragma unroll
  for (int u = 0; u < kColChunk; ++u) {
    a0 += x[u] * ft[3 * (cb + u)];
    a1 += x[u] * ft[3 * (cb + u) + 1];
    a2 += x[u] * ft[3 * (cb + u) + 2];
  }
}
DEV void fwd_col_item(const DevMesh& d, const SweepItem& it, double* ft) {
  const int w = it.w, h = it.h, col0 = it.col0, r0 = it.first & ~kItemColBit;
  const int lane = threadIdx.x & 63;
  const int r = r0 + lane;
  const int nc = r < h ? min(r + 1, w) : 0;
  const int rr = min(r, h - 1);
  const double* blk = d.tvals + it.valoff;
  double xa[kColChunk], xb[kColChunk];
  col_chunk(blk, h, w, rr, nc, 0, xa);
  double b0 = 0, b1 = 0, b2 = 0;
  int32_t orow = 0;
  if (r < h && r >= w) {
    orow = d.dst[it.rowoff + r - w];
    gather_updates(d, it, r, b0, b1, b2);
  }
  // frontal vector; zero past `need` up to the end of the last chunk, so the
  // zero entries of a partial chunk multiply zeros
  const int need = min(w, r0 + kColRows);
  const int ceil_need = (need + kColChunk - 1) / kColChunk * kColChunk;
  for (int c = lane; c < ceil_need; c += 64) {
    double a0 = 0, a1 = 0, a2 = 0;
    if (c < need) {
      a0 = d.rhs[3 * (col0 + c)];
      a1 = d.rhs[3 * (col0 + c) + 1];
      a2 = d.rhs[3 * (col0 + c) + 2];
      gather_updates(d, it, c, a0, a1, a2);
    }
    ft[3 * c] = a0;
    ft[3 * c + 1] = a1;
    ft[3 * c + 2] = a2;
  }
  // the wave's own LDS writes, visible to all of its lanes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (r >= h) return;
  // the chunk loop runs to `need` for the whole wave (uniform column index;
  // a lane's entries past its own nc load as zeros)
  double a0 = 0, a1 = 0, a2 = 0;
  for (int c = 0;;) {
    if (c + kColChunk < need) col_chunk(blk, h, w, rr, nc, c + kColChunk, xb);
    col_fma(xa, ft, c, a0, a1, a2);
    c += kColChunk;
    if (c >= need) break;
    if (c + kColChunk < need) col_chunk(blk, h, w, rr, nc, c + kColChunk, xa);
    col_fma(xb, ft, c, a0, a1, a2);
    c += kColChunk;
    if (c >= need) break;
  }
  if (r < w) {
    d.ybuf[3 * (col0 + r)] = a0;
    d.ybuf[3 * (col0 + r) + 1] = a1;
    d.ybuf[3 * (col0 + r) + 2] = a2;
  } else {
    double* o = d.slots + 3 * (int64_t)orow;
    o[0] = b0 - a0;
    o[1] = b1 - a1;
    o[2] = b2 - a2;
  }
}
// A workgroup of column-form items: wave k takes item base + k if it is in
// the level (ft: kColW * 3 doubles per wave).
DEV void fwd_col_group(const DevMesh& d, int base, int end, double* ft) {
  // the wave index is uniform across the wave: with readfirstlane the item and
  // the block base live in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if (base + wave >= end) return;
  const SweepItem it = d.fwd_items[base + wave];
  fwd_col_item(d, it, ft + wave * kColW * 3);
}

template <int CH>
DEV void b_fwd_t(const DevMesh& d, int bid, int check_done) {
  // the item and the stop flag are read in the same scalar round trip (the
  // empty asm statement keeps the compiler from sinking the item load below
  // the flag test)
  const SweepItem it = d.fwd_items[bid];
  const int done = check_done ? d.ctl->done : 0;
  __asm__ volatile("" ::"s"(it.first), "s"(done));
  if (done) return;
  __shared__ double ft[CH * 3];
  if constexpr (CH == kVecChunk) {
    // column-form items reach this body only through the batched launch,
    // whose map holds the first item of each group of four
    static_assert(CH >= 4 * kColW, "column items share the vector chunk");
    if (it.first & kItemColBit) {
      fwd_col_group(d, bid, it.end, ft);
      return;
    }
    if (it.first & kItemWide) {
      fwd_item<32, CH>(d, it, it.first & ~kItemWide, ft);
      return;
    }
  }
  fwd_item<8, CH>(d, it, it.first, ft);
}
DEV void b_fwd(const DevMesh& d, int bid, int check_done) { b_fwd_t<kVecChunk>(d, bid, check_done); }
// consecutive items of a level mostly belong to one supernode and read the
// same input vector: keep them on one XCD
__global__ void __launch_bounds__(kBlock) k_fwd(DevMesh d, int it0, int check_done) {
  b_fwd(d, it0 + xcd_block((int)blockIdx.x, (int)gridDim.x), check_done);
}
__global__ void __launch_bounds__(kBlock, 8) k_fwd_narrow(DevMesh d, int it0, int check_done) {
  b_fwd_t<kVecChunkNarrow>(d, it0 + xcd_block((int)blockIdx.x, (int)gridDim.x), check_done);
}
// column-form level: workgroup b takes items it0 + 4 b .. it0 + 4 b + 3 (two
// chunks of block entries in flight need more than the 64 registers of eight
// waves per SIMD)
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_fwd_col(DevMesh d, int it0, int it1, int check_done) {
  if (check_done && d.ctl->done) return;
  __shared__ double ft[4 * kColW * 3];
  fwd_col_group(d, it0 + 4 * xcd_block((int)blockIdx.x, (int)gridDim.x), it1, ft);
}

// Backward sweep of one level with the transposed blocks.  Work item (s, c0):
// columns [c0, c0 + 256/LPR) of supernode s.  With z = [y_s; -x[rows]],
//   x_c = sum_{r >= c} L^{-T}-block[c][r - c] z[r].
template <int LPR, int CH>
DEV void bwd_item(const DevMesh& d, const SweepItem& it, int c0, double* x, double* z) {
  const int w = it.w, h = it.h, col0 = it.col0;
  const int t = threadIdx.x;
  const int ncols = min(256 / LPR, w - c0);
  const int32_t* rows = d.rows + it.rowoff;
  double acc[3] = {0, 0, 0};
  for (int vb = c0; vb < h; vb += CH) {
    const int vl = min(CH, h - vb);
    __syncthreads();
    for (int k = t; k < vl; k += kBlock) {
      const int r = vb + k;
      if (r < w) {
        z[3 * k] = d.ybuf[3 * (col0 + r)];
        z[3 * k + 1] = d.ybuf[3 * (col0 + r) + 1];
        z[3 * k + 2] = d.ybuf[3 * (col0 + r) + 2];
      } else {
        const int32_t g = rows[r - w];
        z[3 * k] = -x[3 * g];
        z[3 * k + 1] = -x[3 * g + 1];
        z[3 * k + 2] = -x[3 * g + 2];
      }
    }
    __syncthreads();
    row_products<false, LPR>(d.tvals, it.valoff, w, h, c0, ncols, z, vb, vl, acc);
  }
  const int lane = t & 63, wave = t >> 6, g = lane / LPR, l = lane % LPR;
  const int cc = wave * (64 / LPR) + g;
  if (l == 0 && cc < ncols) {
    const int c = c0 + cc;
    x[3 * (col0 + c)] = acc[0];
    x[3 * (col0 + c) + 1] = acc[1];
    x[3 * (col0 + c) + 2] = acc[2];
  }
}
template <int CH>
DEV void b_bwd_t(const DevMesh& d, int bid, double* x, int check_done) {
  const SweepItem it = d.bwd_items[bid];
  const int done = check_done ? d.ctl->done : 0;
  __asm__ volatile("" ::"s"(it.first), "s"(done));
  if (done) return;
  __shared__ double z[CH * 3];
  if constexpr (CH == kVecChunk) {
    if (it.first & kItemWide) {
      bwd_item<32, CH>(d, it, it.first & ~kItemWide, x, z);
      return;
    }
  }
  bwd_item<8, CH>(d, it, it.first, x, z);
}
DEV void b_bwd(const DevMesh& d, int bid, double* x, int check_done) { b_bwd_t<kVecChunk>(d, bid, x, check_done); }
__global__ void __launch_bounds__(kBlock) k_bwd(DevMesh d, int it0, double* x, int check_done) {
  b_bwd(d, it0 + xcd_block((int)blockIdx.x, (int)gridDim.x), x, check_done);
}
__global__ void __launch_bounds__(kBlock, 8) k_bwd_narrow(DevMesh d, int it0, double* x, int check_done) {
  b_bwd_t<kVecChunkNarrow>(d, it0 + xcd_block((int)blockIdx.x, (int)gridDim.x), x, check_done);
}

// One level of each sweep, narrow or wide variant as the plan marks it.
static void launch_fwd_level(const DevMesh& d, const SolvePlan& pl, int L, int check_done, hipStream_t st) {
  const int n0 = pl.fwd_ptr[L], n1 = pl.fwd_ptr[L + 1];
  if (n1 <= n0) return;
  if (pl.fwd_col[L]) hipLaunchKernelGGL(k_fwd_col, dim3((n1 - n0 + 3) / 4), dim3(kBlock), 0, st, d, n0, n1, check_done);
  else if (pl.fwd_narrow[L]) hipLaunchKernelGGL(k_fwd_narrow, dim3(n1 - n0), dim3(kBlock), 0, st, d, n0, check_done);
  else hipLaunchKernelGGL(k_fwd, dim3(n1 - n0), dim3(kBlock), 0, st, d, n0, check_done);
}
static void launch_bwd_level(const DevMesh& d, const SolvePlan& pl, int k, double* x, int check_done,
                             hipStream_t st) {
  const int n0 = pl.bwd_ptr[k], n1 = pl.bwd_ptr[k + 1];
  if (n1 <= n0) return;
  if (pl.bwd_narrow[k]) hipLaunchKernelGGL(k_bwd_narrow, dim3(n1 - n0), dim3(kBlock), 0, st, d, n0, x, check_done);
  else hipLaunchKernelGGL(k_bwd, dim3(n1 - n0), dim3(kBlock), 0, st, d, n0, x, check_done);
}

// q = solution at free vertices, pin targets at pinned vertices
__global__ void __launch_bounds__(kBlock) k_set_pins(DevMesh d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.npins) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) d.q[3 * (d.nf + i) + c] = d.pin_xyz[3 * i + c];
}

DEV void b_add_q(const DevMesh& d, int bid) {
  int i = bid * blockDim.x + threadIdx.x;
  if (stopped(d, i < 3 * d.nf ? d.dq[i] : 0.0)) return;
  const double sg = d.ctl->sigma;
  if (i >= 3 * d.nf) return;
  d.q[i] += sg * d.dq[i];
}
__global__ void __launch_bounds__(kBlock) k_add_q(DevMesh d) { b_add_q(d, blockIdx.x); }

// Accept a step at element i: X = S + sigma D(p) (plus R^T Zc_i, a world-frame
// field such as the contact step, with kZc), R <- R polar(X) (re-orthonormalized),
// S <- polar(X)^T X; R and S are updated in memory and in place.
template <bool kZc>
DEV void accept_elem(const DevMesh& d, int i, double sigma, const double* zc, double (&R)[9], double (&S)[9]) {
  const int m = d.m;
  double py[9], D[9], X[9], Rx[9], Rn[9], Sn[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) py[k] = d.p[k * m + i];
  from_y<double>(py, D);
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = S[k] + sigma * D[k];
  if constexpr (kZc) {
    double Z[9], RZ[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Z[k] = zc[k * m + i];
    matTmul3(R, Z, RZ);
#pragma unroll
    for (int k = 0; k < 9; ++k) X[k] += RZ[k];
  }
  if (!polar3_newton(X, Rx)) {
    const Mat3 r = polar3_fallback(load_mat3(X));
#pragma unroll
    for (int k = 0; k < 9; ++k) Rx[k] = r.v[k];
  }
  matmul3(R, Rx, Rn);
  reorthonormalize(Rn);
  matTmul3(Rx, X, Sn);
  double sy[9];
  to_y<double, double>(Sn, sy);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    R[k] = Rn[k];
    d.R[k * m + i] = Rn[k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) d.S[k * m + i] = sy[k];
  s_from6(sy, S);
}

// --------------------------------------------------------------- element pass
// The element pass at element i: the accept of the pending step (sigma > 0),
// then at the new state the energy term (added to acc[0]), inverted-tet
// count, and the exact gradient in y coordinates gy with its squared norm gn.
// S is the stretch after the accept.
DEV void element_core(const DevMesh& d, int i, double sigma, Elem& e, double (&S)[9], double (&gy)[9], double& gn,
                      DD (&acc)[2], int& ninv) {
  load_elem(d, i, e);
  double R[9];
  load_R(d, i, R);
  load_S(d, i, S);
  if (sigma != 0.0) accept_elem<false>(d, i, sigma, nullptr, R, S);
  double A[9], At[9];
  gather_grad(d.q, e, A);
  matTmul3(R, A, At);
  const double beta = d.alpha * e.w;
  const double J = det3(S);
  double C[9];
  cof3<double>(S, C);
  double Su[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) Su[c] = S[3 * c] * e.u[0] + S[3 * c + 1] * e.u[1] + S[3 * c + 2] * e.u[2];
  double trSS = 0, dres = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    trSS += S[k] * S[k];
    dres += (At[k] - S[k]) * (At[k] - S[k]);
  }
  const double afk = e.a * d.kf;
  const double psi = 0.5 * e.mu * (trSS - 3.0) - e.mu * (J - 1.0) + 0.5 * e.lhat * (J - 1.0) * (J - 1.0) +
                     afk * (Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2]);
  // external work (Sec. 3.4): f . q*(F) = sum_i nu_i . F_i + const with
  // nu_i = w_i G_i L_ff^{-1} f; in the rotated frame nu_rot = R^T nu
  double nur[9];
  if (d.has_ext) {
    double nu[9];
    gather_grad(d.vext, e, nu);
    matTmul3(R, nu, nur);
#pragma unroll
    for (int k = 0; k < 9; ++k) nur[k] *= e.w;
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) nur[k] = 0.0;
  }
  double wext = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) wext += nur[k] * S[k];
  acc[0] = dd_add_d(acc[0], e.vol * psi + 0.5 * beta * dres - wext);
  ninv += (J <= 0.0);
  const double kap = e.lhat * (J - 1.0) - e.mu;
  double G[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      G[3 * a + b] = e.vol * (e.mu * S[3 * a + b] + kap * C[3 * a + b] + 2.0 * afk * Su[a] * e.u[b]) +
                     beta * (S[3 * a + b] - At[3 * a + b]) - nur[3 * a + b];
  gn = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) gn += G[k] * G[k];
  to_y<double, double>(G, gy);
}

// Accept the previous step (if sigma > 0): X = S + sigma D(p), R <- R polar(X),
// S <- sym(polar(X)^T X).  Then at the new state: energy, exact gradient
// G = vol P(F) + beta (F - A) (eq. gradient), the two clamped Hessian blocks
// + beta I, their inverses and gbar = H^{-1} g.
template <typename T>
DEV void b_element(const DevMesh& d, int bid) {
  Ctl* ctl = d.ctl;
  {
    const int i0 = xcd_block(bid, d.nb) * kBlock + threadIdx.x;
    if (stopped(d, i0 < d.m ? d.vol[i0] : 0.0)) return;
  }
  __shared__ DD sh[2 * kBlock];
  __shared__ int shc[kBlock];
  const double sigma = ctl->sigma;
  DD acc[2] = {DD{0, 0}, DD{0, 0}};
  int ninv = 0;
  const int m = d.m;
  for (int i = xcd_block(bid, d.nb) * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    Elem e;
    double S[9], gy[9], gn;
    element_core(d, i, sigma, e, S, gy, gn, acc, ninv);
    const int bpos = d.nbones ? d.bone_pos[i] : -1;
    if (bpos < 0) {
      acc[1] = dd_add_d(acc[1], gn);
      T* gyo = (T*)d.gbar;
#pragma unroll
      for (int k = 0; k < 9; ++k) gyo[k * m + i] = (T)gy[k];
    } else {
      // affine bone tet: its gradient is a term of the bone's (k_bone_blocks)
#pragma unroll
      for (int k = 0; k < 9; ++k) d.bone_gbuf[(int64_t)k * d.nbt + bpos] = gy[k];
    }
  }
  block_reduce_dd<2>(acc, sh);
  const int ninv_sum = block_sum_int(ninv, shc);
  if (threadIdx.x == 0) {
    d.part_e[2 * bid] = acc[0].hi;
    d.part_e[2 * bid + 1] = acc[0].lo;
    d.part_g[2 * bid] = acc[1].hi;
    d.part_g[2 * bid + 1] = acc[1].lo;
    d.part_cnt[2 * bid + 1] = ninv_sum;
  }
}

// Hessian blocks of the element pass: at the state left by b_element, the two
// clamped blocks + beta I in the rotated basis (precision T), their inverses
// (from their Cholesky factors), and gbar = H^{-1} g (g read from gbar,
// overwritten in place).  The inverses are stored, not the factors: the Gram
// pass needs them explicitly, and applying one is a matrix-vector product.
// The two blocks at a stretch S with material scalars (vol mu, vol lhat,
// a k_f): the element's own, or a bone's sums over its tets (the Hessian is
// linear in vol mu and vol lhat at a fixed S).
template <typename T>
DEV void hess_blocks_s(const double* S, double vmu, double vlhat, double vafk, const double* u, T (&Hs)[6][6],
                       T (&Hk)[3][3]) {
  const double J = det3(S);
  double C[9];
  cof3<double>(S, C);
  const double vkap = vlhat * (J - 1.0) - vmu;
  T St[9], ut[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) St[k] = (T)S[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) ut[k] = (T)u[k];
  const T muT = (T)vmu, kapT = (T)vkap, phiT = (T)(2.0 * vafk), lhT = (T)vlhat;
  T cy[9];
  to_y<T, double>(C, cy);
#pragma unroll
  for (int y = 0; y < 6; ++y)
#pragma unroll
    for (int z = 0; z < 6; ++z) Hs[y][z] = hproj<T>(y, z, St, muT, kapT, phiT, ut) + lhT * cy[y] * cy[z];
#pragma unroll
  for (int y = 0; y < 3; ++y)
#pragma unroll
    for (int z = 0; z < 3; ++z) Hk[y][z] = hproj<T>(6 + y, 6 + z, St, muT, kapT, phiT, ut);
}

template <typename T>
DEV void hess_blocks(const DevMesh& d, int i, T (&Hs)[6][6], T (&Hk)[3][3], bool fiber = true) {
  const int m = d.m;
  double S[9];
  load_S(d, i, S);
  const double vol = d.vol[i];
  double u[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u[c] = d.fib[c * m + i];
  const int g = d.grp[i];
  const double afk = fiber ? (g >= 0 ? d.act[g] : 0.0) * d.kf : 0.0;
  hess_blocks_s<T>(S, vol * d.mu[i], vol * d.lhat[i], vol * afk, u, Hs, Hk);
}

// The two blocks of element i clamped to their positive semi-definite part,
// beta I added, factored and inverted into Lf, with gbar = H^{-1} g.  g: the
// gradient in y coordinates (precision T), or null to read it from gbar.  A
// 6x6 block that is not positive definite (rare) is parked, lower triangle,
// in its inverse's place with its part of g in gbar, and listed in fix for
// lane 0 of the wave.
template <typename T>
DEV void hess_finish(const DevMesh& d, int i, T (&Hs)[6][6], T (&Hk)[3][3], T beta, const T* g, int* fix, int& nfix,
                     int& nclamp) {
  const int m = d.m;
  T* gbar = (T*)d.gbar;
  T* Lf = (T*)d.Lf;
  {
    T Ls[21];
    if (chol_packed<T, 6>(Hs, Ls)) {
      T rds[6];
      add_factor<T, 6>(Hs, beta, Ls, rds);
      T gs[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) gs[k] = g ? g[k] : gbar[k * m + i];
      chol_inverse_apply_store<T, 6>(Ls, rds, gs, Lf, m, i);
#pragma unroll
      for (int k = 0; k < 6; ++k) gbar[k * m + i] = gs[k];
    } else {
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) Lf[(r * (r + 1) / 2 + c) * m + i] = Hs[r][c];
      if (g)
#pragma unroll
        for (int k = 0; k < 6; ++k) gbar[k * m + i] = g[k];
      fix[atomicAdd(&nfix, 1)] = i;
    }
  }
  T Lk[6], rdk[3];
  nclamp += clamp_add_factor<T, 3>(Hk, beta, Lk, rdk);
  T gk[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gk[k] = g ? g[6 + k] : gbar[(6 + k) * m + i];
  chol_inverse_apply_store<T, 3>(Lk, rdk, gk, Lf + (int64_t)21 * m, m, i);
#pragma unroll
  for (int k = 0; k < 3; ++k) gbar[(6 + k) * m + i] = gk[k];
}
// An affine bone tet: identity blocks and gbar = 0, so that the Gram pass
// (which gives it weight 0) reads finite values; k_bone_blocks then stores
// the bone's own block at its first tet.
template <typename T>
DEV void hess_bone_tet(const DevMesh& d, int i) {
  const int m = d.m;
  T* gbar = (T*)d.gbar;
  T* Lf = (T*)d.Lf;
#pragma unroll
  for (int k = 0; k < 27; ++k) Lf[k * m + i] = (k < 21 ? (k == 0 || k == 2 || k == 5 || k == 9 || k == 14 || k == 20)
                                                        : (k == 21 || k == 23 || k == 26)) ? T(1) : T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) gbar[k * m + i] = T(0);
}
// Lane 0 of a wave finishes its wave's indefinite 6x6 blocks: the Jacobi
// clamp in LDS, beta I, the inverse, and gbar = H^{-1} g.
template <typename T>
DEV void hess_fix_list(const DevMesh& d, const int* fix, int nfix, T (&fixW)[6][6], T (&fixV)[6][6], int& nclamp) {
  const int m = d.m;
  T* gbar = (T*)d.gbar;
  T* Lf = (T*)d.Lf;
  for (int q = 0; q < nfix; ++q) {
    const int j = fix[q];
#pragma unroll 1
    for (int r = 0; r < 6; ++r)
#pragma unroll 1
      for (int c = 0; c <= r; ++c) fixW[r][c] = fixW[c][r] = Lf[(r * (r + 1) / 2 + c) * m + j];
    clamp_psd_jacobi_lds<T, 6>(fixW, fixV);
    T Ls[21], Ps[21];
    add_factor<T, 6>(fixW, (T)(d.alpha * d.w[j]), Ls);
    chol_inverse<T, 6>(Ls, Ps);
    T gs[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gs[k] = gbar[k * m + j];
    sym_apply<T, 6>(Ps, gs);
#pragma unroll
    for (int k = 0; k < 6; ++k) gbar[k * m + j] = gs[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) Lf[k * m + j] = Ps[k];
    ++nclamp;
  }
}

// Both blocks are clamped to their positive semi-definite part, beta I is
// added and the results inverted; gbar = H^{-1} g in place.  The elements of
// a workgroup are taken in rounds of kBlock; a 6x6 block that is not positive
// definite (rare) is parked, lower triangle, in its inverse's place and
// finished after the round by lane 0 of its wave with an LDS-resident Jacobi,
// so that the eigen-decomposition holds no registers in the main loop.  The
// fix lists are per wave, so the rounds need no workgroup barrier and a
// wave's next loads are not held up by the other waves' arithmetic.
// Between the waves' own steps: their stores (the parked blocks in Lf)
// visible to lane 0, whose loads come after.
DEV void wave_sync_mem() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
template <typename T, bool kC = false>
DEV void b_element_hess(const DevMesh& d, int bid) {
  const int lb = xcd_block(bid, d.nb);
  {
    const int i0 = lb * kBlock + threadIdx.x;
    if (stopped(d, i0 < d.m ? d.vol[i0] : 0.0)) return;
  }
  constexpr int kW = kBlock / 64;
  __shared__ int shc[kBlock];
  __shared__ int fixl[kW][64];
  __shared__ int nfixw[kW];
  __shared__ T fixWw[kW][6][6], fixVw[kW][6][6];
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  int* fix = fixl[wave];
  int& nfix = nfixw[wave];
  T(&fixW)[6][6] = fixWw[wave];
  T(&fixV)[6][6] = fixVw[wave];
  int nclamp = 0;
  const int m = d.m;
  for (int base = lb * kBlock; base < m; base += d.nb * kBlock) {
    if (lane == 0) nfix = 0;
    wave_sync_mem();
    const int i = base + threadIdx.x;
    const bool own = i < m && !(d.nbones && d.bone_pos[i] >= 0);  // bone tets: k_bone_blocks
    if (own) {
      T Hs[6][6], Hk[3][3];
      hess_blocks<T>(d, i, Hs, Hk, !kC);
      hess_finish<T>(d, i, Hs, Hk, (T)(d.alpha * d.w[i]), nullptr, fix, nfix, nclamp);
    } else if (i < m) {
      hess_bone_tet<T>(d, i);
    }
    wave_sync_mem();
    if (lane == 0) hess_fix_list<T>(d, fix, nfix, fixW, fixV, nclamp);
    if constexpr (kC) {
      wave_sync_mem();
      if (own) coupled_finish<T>(d, i);
    }
    // nfix and fix are reused by the next round
    wave_sync_mem();
  }
  const int nclamp_sum = block_sum_int(nclamp, shc);
  if (threadIdx.x == 0) d.part_cnt[2 * bid] = nclamp_sum;
}
template <typename T>
__global__ void __launch_bounds__(kBlock) k_element(DevMesh d) { b_element<T>(d, blockIdx.x); }
template <typename T, bool kC = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_element_hess(DevMesh d) { b_element_hess<T, kC>(d, blockIdx.x); }


// --------------------------------------------------------------- Woodbury Gram
// Per element: Z = T H^{-1} T^T (9x9, F coordinates; T = (R (x) I) Y) and the
// mode gradients gphi_j = sum_v phi_j(v) b_v.  Accumulates, per workgroup,
//   Gram[(c,j),(c',j')] += w^2 gphi_j^T Z_{cc'} gphi_j'   (6 pairs c <= c')
//   y[(c,j)]            += w (R D(gbar) gphi_j)[c]
// Each wave owns a contiguous run of elements.  Phase A: one lane per element
// (batches of kGramBatch) forms the six 3x3 coordinate-pair blocks of Z, R D(gbar),
// w and the 16 mode gradients into the wave's LDS rows.  Phase B: for each
// pair block, 16x16x4 matrix-core products whose K index runs over the
// batch's (element e, coordinate k) pairs, four per product; lane
// (j, s) = (l % 16, l / 16) supplies A = w_e^2 gphi_j[k] and
// B = (Z_{cc'} gphi_j)[k] for the pair in K slot s.  Waves are added in a
// fixed order at the end.
constexpr int kGramBatch = 16;
// FP64 steps of a full batch's product loop unrolled together (4: same time,
// 3: slower, 12: spills; the loop of runtime length did not unroll at all)
constexpr int kGramUnroll = 2;
constexpr int kGramRow = 65;   // 54 block entries + 9 + 1, padded to an odd stride
constexpr int kGramGRow = 49;  // 16 mode gradients x 3, padded

template <typename T>
struct MfmaAcc;
// 16x16x4 products; A[i][k] comes from lane i + 16 k, B[k][j] from lane j + 16 k,
// and register r of lane l holds D[row(l, r)][l % 16] (the FP64 and FP32
// forms distribute the rows differently).
template <>
struct MfmaAcc<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static DEV v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static DEV int row(int l, int r) { return 4 * r + (l >> 4); }
};
template <>
struct MfmaAcc<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static DEV v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static DEV int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// Z blocks of one element (phase A): zr[p * 9 + a * 3 + b] = Z[3c + a][3c' + b]
// for the pairs p = (0,0) (0,1) (0,2) (1,1) (1,2) (2,2), from the element's
// rotation R and its stored block inverses (Hs: 6x6, Hk: 3x3, packed lower;
// Hf: the coupled 9x9 inverse, kC only).  The lane computes the entries whose
// first F coordinate is c (c = 0, 1, 2: three lanes per element share the
// work; c = 3 computes and stores nothing useful).
template <typename T, bool kC>
DEV void gram_zmath(const T* Rp, const T* Hs, const T* Hk, const T* Hf, int c, T* zr) {
  // the lane picks a row of R below: from a local copy, not from the caller's
  // array (a pick from that array becomes a load from a chosen address and
  // keeps the array in scratch memory)
  T R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = Rp[k];
  // per gradient-direction pair (dd <= dp): M[e][e'] = (Y H^{-1} Y^T)[(e,dd),(e',dp)],
  // then Z[(c,dd),(c',dp)] = (R M R^T)[c][c'], stored in the block of (min, max)(c, c')
  const int cr = c < 2 ? c : 2;
  const T Rc[3] = {cr == 0 ? R[0] : (cr == 1 ? R[3] : R[6]), cr == 0 ? R[1] : (cr == 1 ? R[4] : R[7]),
                   cr == 0 ? R[2] : (cr == 1 ? R[5] : R[8])};
#pragma unroll
  for (int dd = 0; dd < 3; ++dd)
#pragma unroll
    for (int dp = dd; dp < 3; ++dp) {
      T Mx[3][3];
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int ep = 0; ep < 3; ++ep) {
          const int A = 3 * e + dd, B = 3 * ep + dp;
          T v = 0;
#pragma unroll
          for (int pa = 0; pa < 2; ++pa)
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) {
              const int ya = kYof[A][pa], yb = kYof[B][pb];
              if constexpr (kC) {
                if (ya >= 0 && yb >= 0) {
                  const int lo = ya < yb ? ya : yb, hi = ya < yb ? yb : ya;
                  v += T(kYvf[A][pa] * kYvf[B][pb]) * Hf[hi * (hi + 1) / 2 + lo];
                }
                continue;
              }
              if (ya >= 0 && yb >= 0 && (ya < 6) == (yb < 6)) {
                const T cv = T(kYvf[A][pa] * kYvf[B][pb]);
                if (ya < 6) {
                  const int lo = ya < yb ? ya : yb, hi = ya < yb ? yb : ya;
                  v += cv * Hs[hi * (hi + 1) / 2 + lo];
                } else {
                  const int lo = (ya < yb ? ya : yb) - 6, hi = (ya < yb ? yb : ya) - 6;
                  v += cv * Hk[hi * (hi + 1) / 2 + lo];
                }
              }
            }
          Mx[e][ep] = v;
        }
      T RM[3];
#pragma unroll
      for (int ep = 0; ep < 3; ++ep) RM[ep] = Rc[0] * Mx[0][ep] + Rc[1] * Mx[1][ep] + Rc[2] * Mx[2][ep];
#pragma unroll
      for (int cp = 0; cp < 3; ++cp) {
        const T v = RM[0] * R[3 * cp] + RM[1] * R[3 * cp + 1] + RM[2] * R[3 * cp + 2];
        // v = Z[3c + dd][3cp + dp]; for dd == dp the entries with cp < c
        // are those of the lane of row cp
        if (c > 2 || (dd == dp && cp < c)) continue;
        if (c <= cp) {
          const int p = c == 0 ? cp : (c == 1 ? 2 + cp : 5);
          zr[p * 9 + dd * 3 + dp] = v;
          if (dd != dp && c == cp) zr[p * 9 + dp * 3 + dd] = v;
        } else {
          const int p = cp == 0 ? c : (cp == 1 ? 2 + c : 5);
          zr[p * 9 + dp * 3 + dd] = v;
        }
      }
    }
}

// The same for element i, reading R and the block inverses from memory.
template <typename T, bool kC = false>
DEV void gram_zblocks(const DevMesh& d, int i, int c, T* zr) {
  const int m = d.m;
  T R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = (T)d.R[k * m + i];
  const T* Lf = (const T*)d.Lf;
  // the stored block inverses D^{-1} (6x6 and 3x3, packed lower)
  T Hs[21], Hk[6];
#pragma unroll
  for (int k = 0; k < 21; ++k) Hs[k] = Lf[k * m + i];
#pragma unroll
  for (int k = 0; k < 6; ++k) Hk[k] = Lf[(21 + k) * m + i];
  // coupled form: the full inverse blockdiag(D^{-1}) - W K^{-1} W^T in the
  // rotated (y) coordinates, packed lower, W = D^{-1} V
  [[maybe_unused]] T Hf[kC ? 45 : 1];
  if constexpr (kC) {
    T V[9][3], W[9][3];
    fiber_V<T>(d, i, V);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        T v = 0;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
          if ((a < 6) != (b < 6)) continue;
          T h;
          if (a < 6) h = Hs[(a > b ? a : b) * ((a > b ? a : b) + 1) / 2 + (a > b ? b : a)];
          else h = Hk[(a > b ? a - 6 : b - 6) * ((a > b ? a - 6 : b - 6) + 1) / 2 + (a > b ? b - 6 : a - 6)];
          v += h * V[b][cc];
        }
        W[a][cc] = v;
      }
    // K^{-1}, stored packed
    T Ki[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc <= r; ++cc) Ki[r][cc] = Ki[cc][r] = Lf[(kLfSplit + r * (r + 1) / 2 + cc) * m + i];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      T u0 = W[a][0] * Ki[0][0] + W[a][1] * Ki[1][0] + W[a][2] * Ki[2][0];
      T u1 = W[a][0] * Ki[0][1] + W[a][1] * Ki[1][1] + W[a][2] * Ki[2][1];
      T u2 = W[a][0] * Ki[0][2] + W[a][1] * Ki[1][2] + W[a][2] * Ki[2][2];
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        T h = T(0);
        if (a < 6 && b < 6) h = Hs[a * (a + 1) / 2 + b];
        else if (a >= 6 && b >= 6) h = Hk[(a - 6) * (a - 5) / 2 + (b - 6)];
        Hf[a * (a + 1) / 2 + b] = h - (u0 * W[b][0] + u1 * W[b][1] + u2 * W[b][2]);
      }
    }
  }
  gram_zmath<T, kC>(R, Hs, Hk, Hf, c, zr);
}

// Broadcast within a quad of lanes: every lane gets lane K's value.
template <int K>
DEV double quad_bcast(double x) {
  constexpr int ctrl = K * 0x55;  // quad_perm [K, K, K, K]
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int K>
DEV float quad_bcast(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), K * 0x55, 0xF, 0xF, true));
}
template <typename U>
DEV U quad_from(U x, int k) {
  switch (k) {
    case 0: return quad_bcast<0>(x);
    case 1: return quad_bcast<1>(x);
    case 2: return quad_bcast<2>(x);
    default: return quad_bcast<3>(x);
  }
}

// Phase A inputs of one element (split blocks), loaded one batch ahead of
// their use and spread over the element's four lanes: lane s holds rows
// s, s + 4, ... of each per-element array (R, the stored block inverses,
// gbar, D_m^{-1}); the quad broadcasts them when the batch is formed.  The
// vertex ids are loaded one batch earlier still, so that the mode-gradient
// gather that depends on them is issued together with the rest.
template <typename T>
struct GramPart {
  T R[3], Lf[7], gb[3];
  double bm[3];
  T w;
};
template <typename T>
DEV void gram_load_part(const DevMesh& d, int i, int s, GramPart<T>& g) {
  const int m = d.m;
  const T* Lf = (const T*)d.Lf;
  const T* gbar = (const T*)d.gbar;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int r = min(s + 4 * u, 8);  // rows past the end repeat row 8 (unused)
    g.R[u] = (T)d.R[r * m + i];
    g.gb[u] = gbar[r * m + i];
    g.bm[u] = d.dminv[r * m + i];
  }
#pragma unroll
  for (int u = 0; u < 7; ++u) g.Lf[u] = Lf[min(s + 4 * u, 26) * m + i];
  // affine bone tets enter through their bone's row (k_bone_blocks)
  g.w = (d.nbones && d.bone_pos[i] >= 0) ? T(0) : (T)d.w[i];
}
DEV void gram_load_vid(const DevMesh& d, int i, int32_t (&vid)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) vid[v] = d.vid[v * d.m + i];
}
// modes q4 .. q4 + 3 of the element's four vertices
DEV void gram_load_phi(const DevMesh& d, const int32_t (&vid)[4], int q4, double (&ph)[4][4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double2* p = reinterpret_cast<const double2*>(d.phi + (int64_t)kMaxK1 * vid[v] + q4);
    const double2 p0 = p[0], p1 = p[1];
    ph[v][0] = p0.x;
    ph[v][1] = p0.y;
    ph[v][2] = p1.x;
    ph[v][3] = p1.y;
  }
}
// Phase A of one element from the quad's registers: lane sl writes its Z
// entries and row sl of R D(gbar) (sl < 3) or w (sl = 3), and mode
// gradients 4 sl .. 4 sl + 3.
template <typename T>
DEV void gram_phase_a(const GramPart<T>& g, const double (&ph)[4][4], int sl, int k1, T* zr, T* gr) {
  T R[9], Hs[21], Hk[6];
#pragma unroll
  for (int r = 0; r < 9; ++r) R[r] = quad_from(g.R[r / 4], r % 4);
#pragma unroll
  for (int r = 0; r < 27; ++r) {
    const T v = quad_from(g.Lf[r / 4], r % 4);
    if (r < 21) Hs[r] = v;
    else Hk[r - 21] = v;
  }
  gram_zmath<T, false>(R, Hs, Hk, nullptr, sl, zr);
  // gbar and D_m^{-1} after the Z blocks, when their registers are free
  double gbd[9], bm[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    gbd[r] = (double)quad_from(g.gb[r / 4], r % 4);
    bm[r] = quad_from(g.bm[r / 4], r % 4);
  }
  if (sl < 3) {
    double D[9];
    from_y<double>(gbd, D);
    const double r0 = (double)(sl == 0 ? R[0] : (sl == 1 ? R[3] : R[6]));
    const double r1 = (double)(sl == 0 ? R[1] : (sl == 1 ? R[4] : R[7]));
    const double r2 = (double)(sl == 0 ? R[2] : (sl == 1 ? R[5] : R[8]));
#pragma unroll
    for (int q = 0; q < 3; ++q) zr[54 + 3 * sl + q] = (T)(r0 * D[q] + r1 * D[3 + q] + r2 * D[6 + q]);
  } else {
    zr[63] = g.w;
  }
  double b[4][3];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int c = 0; c < 3; ++c) b[v][c] = bm[3 * v + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) b[3][c] = -(b[0][c] + b[1][c] + b[2][c]);
  double gg[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) gg[q][0] = gg[q][1] = gg[q][2] = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) gg[q][c] += ph[v][q] * b[v][c];
  const int q4 = 4 * sl;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) gr[3 * (q4 + q) + c] = q4 + q < k1 ? (T)gg[q][c] : T(0);
}

template <typename T, bool kC = false>
DEV void b_gram(const DevMesh& d, int bid) {
  if (d.ctl->done) return;
  typedef typename MfmaAcc<T>::v4 v4;
  // wave tiles of phase A (Z blocks, R D(gbar), w, mode gradients), reused for
  // the final combination of the waves
  constexpr size_t kTileBytes = sizeof(T) * (kBlock / 64) * kGramBatch * (kGramRow + kGramGRow);
  constexpr size_t kCombBytes = sizeof(double) * 3 * 64 * 25;
  __shared__ double sbuf[((kTileBytes > kCombBytes ? kTileBytes : kCombBytes) + 7) / 8];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  T(*zw)[kGramRow] = reinterpret_cast<T(*)[kGramRow]>(sbuf) + wave * kGramBatch;
  T(*gw)[kGramGRow] =
      reinterpret_cast<T(*)[kGramGRow]>(reinterpret_cast<T*>(sbuf) + (kBlock / 64) * kGramBatch * kGramRow) +
      wave * kGramBatch;
  const int m = d.m;
  const int per = (m + d.nbg - 1) / d.nbg;
  const int e0 = xcd_block(bid, d.nbg) * per, e1 = min(m, e0 + per);
  const int perw = (per + 3) / 4;
  const int w0 = min(e1, e0 + wave * perw), w1 = min(e1, w0 + perw);
  const int k1 = d.k1;
  const int j = lane & 15, k = lane >> 4;
  v4 acc[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) acc[p] = v4{0, 0, 0, 0};
  // y[(c, j)] partials of this lane's K slot k: step st takes pair
  // f = 4 st + k, whose coordinate is (st + k) mod 3 in every batch, so the
  // terms of step st collect in ry[st mod 3] (coordinate (m + k) mod 3 for
  // ry[m]), each in step order
  T ry[3] = {0, 0, 0};
  const int el = lane >> 2, sl = lane & 3;
  // split blocks: the next batch's inputs are requested before this batch's
  // products, so their latency overlaps the matrix-core work
  [[maybe_unused]] GramPart<T> nxt;
  [[maybe_unused]] double ph[4][4];
  [[maybe_unused]] int32_t vid[4];
  if constexpr (!kC) {
    if (el < min(kGramBatch, w1 - w0)) {
      gram_load_vid(d, w0 + el, vid);
      gram_load_part<T>(d, w0 + el, sl, nxt);
      gram_load_phi(d, vid, 4 * sl, ph);
    }
    if (w0 + kGramBatch < w1 && el < min(kGramBatch, w1 - w0 - kGramBatch)) gram_load_vid(d, w0 + kGramBatch + el, vid);
  }
  for (int base = w0; base < w1; base += kGramBatch) {
    const int ne = min(kGramBatch, w1 - base);
    // four lanes per element: lane s = 0, 1, 2 forms the Z entries and the
    // row of R D(gbar) of F coordinate s, lane 3 stores w; each lane forms
    // four of the sixteen mode gradients gphi_j = sum_v phi_j(v) b_v (rows
    // of phi are zero beyond k1 and at pins)
    if constexpr (!kC) {
      if (el < ne) gram_phase_a<T>(nxt, ph, sl, k1, zw[el], gw[el]);
    } else {
      const int q4 = 4 * sl;
      if (el < ne) {
        const int i = base + el;
        gram_zblocks<T, kC>(d, i, sl, zw[el]);
        if (sl < 3) {
          const T* gbar = (const T*)d.gbar;
          double gbd[9], D[9];
#pragma unroll
          for (int q = 0; q < 9; ++q) gbd[q] = (double)gbar[q * m + i];
          from_y<double>(gbd, D);
          const double r0 = (double)(T)d.R[(3 * sl) * m + i], r1 = (double)(T)d.R[(3 * sl + 1) * m + i],
                       r2 = (double)(T)d.R[(3 * sl + 2) * m + i];
#pragma unroll
          for (int q = 0; q < 3; ++q) zw[el][54 + 3 * sl + q] = (T)(r0 * D[q] + r1 * D[3 + q] + r2 * D[6 + q]);
        } else {
          // affine bone tets enter through their bone's row (k_bone_blocks)
          zw[el][63] = (d.nbones && d.bone_pos[i] >= 0) ? T(0) : (T)d.w[i];
        }
        double b[4][3];
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
          for (int c = 0; c < 3; ++c) b[v][c] = d.dminv[(3 * v + c) * m + i];
#pragma unroll
        for (int c = 0; c < 3; ++c) b[3][c] = -(b[0][c] + b[1][c] + b[2][c]);
        double gg[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) gg[q][0] = gg[q][1] = gg[q][2] = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double2* ph = reinterpret_cast<const double2*>(d.phi + (int64_t)kMaxK1 * d.vid[v * m + i] + q4);
          const double2 p0 = ph[0], p1 = ph[1];
          const double pv[4] = {p0.x, p0.y, p1.x, p1.y};
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) gg[q][c] += pv[q] * b[v][c];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) gw[el][3 * (q4 + q) + c] = q4 + q < k1 ? (T)gg[q][c] : T(0);
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if constexpr (!kC) {
      // the next batch's rows and mode gradients (its vertex ids are here
      // already), then the vertex ids of the batch after it
      const int nb = base + kGramBatch, nb2 = nb + kGramBatch;
      if (nb < w1 && el < min(kGramBatch, w1 - nb)) {
        gram_load_part<T>(d, nb + el, sl, nxt);
        gram_load_phi(d, vid, 4 * sl, ph);
      }
      if (nb2 < w1 && el < min(kGramBatch, w1 - nb2)) gram_load_vid(d, nb2 + el, vid);
    }
    // The product loop runs at a raised wave priority: with two waves per
    // SIMD, the wave in its matrix-core loop is issued first and keeps the
    // matrix cores fed, while the other wave's phase A fills the vector ALU
    // in between (alternating runs on one box: FP64 pass 561 -> 546 us, FP32
    // 348 -> 331 us).
    __builtin_amdgcn_s_setprio(1);
    // The K dimension of each product runs over (element, coordinate) pairs
    // of the batch: step st takes the pairs f = 4 st + ks (ks = lane / 16, the
    // lane's K slot) with element f / 3 and coordinate f % 3, so all four
    // slots carry data (twelve products per pair block for sixteen elements
    // instead of sixteen with one slot empty).  A lane's A value (row i) and
    // B value (column j) both belong to its slot's pair.
    // (a full batch runs a loop of constant length, which the compiler can
    // unroll so that one step's LDS reads overlap the previous step's
    // products; the last, partial batch of a wave runs the same body)
    auto step = [&](int st) {
      const int f = 4 * st + k;
      const bool valid = f < 3 * ne;
      const int e = valid ? f / 3 : 0;
      const int kc = valid ? f - 3 * e : 0;
      const T* zr = zw[e];
      const T g0 = gw[e][3 * j], g1 = gw[e][3 * j + 1], g2 = gw[e][3 * j + 2];
      const T wv = valid ? zr[63] : T(0);
      const T gk = kc == 0 ? g0 : (kc == 1 ? g1 : g2);
      const T av = wv * wv * gk;
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const T bv = zr[p * 9 + kc * 3] * g0 + zr[p * 9 + kc * 3 + 1] * g1 + zr[p * 9 + kc * 3 + 2] * g2;
        acc[p] = MfmaAcc<T>::mma(av, bv, acc[p]);
      }
      const T yv = wv * (zr[54 + 3 * kc] * g0 + zr[54 + 3 * kc + 1] * g1 + zr[54 + 3 * kc + 2] * g2);
      const int m = st % 3;
      ry[0] += m == 0 ? yv : T(0);
      ry[1] += m == 1 ? yv : T(0);
      ry[2] += m == 2 ? yv : T(0);
    };
    // Full batch: step 3 i + m (m = 0, 1, 2) takes pair 12 i + 4 m + k,
    // element 4 i + (4 m + k) / 3, so the y term goes to ry[m] without a
    // select.
    auto full_step = [&](int i, auto mc) {
      constexpr int m = decltype(mc)::value;
      const int em = (4 * m + k) / 3, kc = 4 * m + k - 3 * em;
      const T* zr = zw[4 * i + em];
      const T* gr = gw[4 * i + em] + 3 * j;
      const T g0 = gr[0], g1 = gr[1], g2 = gr[2];
      const T wv = zr[63];
      const T gk = kc == 0 ? g0 : (kc == 1 ? g1 : g2);
      const T av = wv * wv * gk;
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const T bv = zr[p * 9 + kc * 3] * g0 + zr[p * 9 + kc * 3 + 1] * g1 + zr[p * 9 + kc * 3 + 2] * g2;
        acc[p] = MfmaAcc<T>::mma(av, bv, acc[p]);
      }
      ry[m] += wv * (zr[54 + 3 * kc] * g0 + zr[54 + 3 * kc + 1] * g1 + zr[54 + 3 * kc + 2] * g2);
    };
    if (ne == kGramBatch) {
      if constexpr (sizeof(T) == 4) {
#pragma unroll 1
        for (int i = 0; i < kGramBatch / 4; ++i) {
          full_step(i, std::integral_constant<int, 0>{});
          full_step(i, std::integral_constant<int, 1>{});
          full_step(i, std::integral_constant<int, 2>{});
        }
      } else {
        // FP64: the three-step rounds need registers this pass does not
        // have at two waves per SIMD (spills: 611 vs 541 us); single steps,
        // two at a time
#pragma unroll kGramUnroll
        for (int st = 0; st < 3 * kGramBatch / 4; ++st) step(st);
      }
    } else {
      const int nst = (3 * ne + 3) / 4;
      for (int st = 0; st < nst; ++st) step(st);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_s_setprio(0);
  }
  // coordinate c of slot k is in ry[(c - k) mod 3]
  const int k3 = k % 3;
  T y0 = k3 == 0 ? ry[0] : (k3 == 1 ? ry[2] : ry[1]);
  T y1 = k3 == 0 ? ry[1] : (k3 == 1 ? ry[0] : ry[2]);
  T y2 = k3 == 0 ? ry[2] : (k3 == 1 ? ry[1] : ry[0]);
  // y[(c, j)]: add the four K slots of mode j (lanes j + 16 ks), then lane
  // j + 16 c (c < 3) holds coordinate c
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
    y0 += __shfl_xor(y0, off);
    y1 += __shfl_xor(y1, off);
    y2 += __shfl_xor(y2, off);
  }
  const T yacc = k == 0 ? y0 : (k == 1 ? y1 : y2);
  // add the waves in a fixed order (0 + 1 + 2 + 3) through LDS, then write
  __syncthreads();
  double* comb = sbuf;
  if (wave > 0) {
    double* o = comb + (size_t)(wave - 1) * 64 * 25;
#pragma unroll
    for (int p = 0; p < 6; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) o[(p * 4 + r) * 64 + lane] = (double)acc[p][r];
    o[24 * 64 + lane] = (double)yacc;
  }
  __syncthreads();
  if (wave == 0) {
    double* out = d.part_gram + (int64_t)kGramEntries * bid;
#pragma unroll
    for (int p = 0; p < 6; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = (double)acc[p][r];
#pragma unroll
        for (int w = 0; w < 3; ++w) v += comb[(size_t)w * 64 * 25 + (p * 4 + r) * 64 + lane];
        out[p * 256 + MfmaAcc<T>::row(lane, r) * 16 + j] = v;
      }
    if (k < 3) {
      double v = (double)yacc;
#pragma unroll
      for (int w = 0; w < 3; ++w) v += comb[(size_t)w * 64 * 25 + 24 * 64 + lane];
      out[1536 + k * 16 + j] = v;
    }
  }
}
// FP32: at most three waves per SIMD.  With 101 VGPRs the compiler allowed
// four, and the pass took 679 us instead of 434 us on the 1.5M-tet hinge limb
// (more element gathers in flight per CU than its caches serve).
template <typename T>
constexpr int gram_max_waves() { return sizeof(T) == 4 ? 3 : 8; }
template <typename T, bool kC>
constexpr int gram_min_waves() { return sizeof(T) == 8 && !kC ? 2 : 1; }
template <typename T, bool kC = false>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(gram_min_waves<T, kC>(), gram_max_waves<T>())))
k_gram(DevMesh d) { b_gram<T, kC>(d, blockIdx.x); }

// Partial Gram sums: 16 threads per entry sum interleaved workgroup partials,
// then add their results in a fixed order.
DEV void b_gram_reduce(const DevMesh& d, int bid) {
  __shared__ double sh[16][17];
  const int t = threadIdx.x, part = t >> 4, el = t & 15;
  const int e = bid * 16 + el;
  if (stopped(d, e < kGramEntries && part < d.nbg ? d.part_gram[(int64_t)part * kGramEntries + e] : 0.0)) return;
  // partials part, part + 16, ... (nbg <= 512: at most 32 per thread), all
  // requested before the first addition; even ones into s0, odd ones into s1
  constexpr int kPer = 512 / 16;
  double v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int b = part + 16 * k;
    v[k] = e < kGramEntries && b < d.nbg ? d.part_gram[(int64_t)b * kGramEntries + e] : 0.0;
  }
  double s0 = 0, s1 = 0;
#pragma unroll
  for (int k = 0; k < kPer; k += 2) {
    s0 += v[k];
    s1 += v[k + 1];
  }
  sh[part][el] = s0 + s1;
  __syncthreads();
  if (part == 0 && e < kGramEntries) {
    double s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += sh[k][el];
    for (int b = 0; b < d.nbones; ++b) s += d.part_gram[(int64_t)(d.nbg + b) * kGramEntries + e];
    d.gram[e] = s;
  }
}
__global__ void __launch_bounds__(kBlock) k_gram_reduce(DevMesh d) { b_gram_reduce(d, blockIdx.x); }

// One workgroup: reduce energy / gradient-norm partials, test convergence,
// build C = Lambda - alpha Gram (3k1 x 3k1) with all threads; then the first
// wave factors it (Cholesky, lane r owns row r in registers, pivot columns
// broadcast by lane shuffles) and solves z = C^{-1} y.
constexpr int kCtlThreads = kBlock;
DEV void b_control_a(const DevMesh& d, int bid) {
  Ctl* ctl = d.ctl;
  if (ctl->done) return;
  __shared__ DD sh[2 * kCtlThreads];
  __shared__ int cnt[2][kCtlThreads];
  __shared__ double Cm[49][49];  // C (48 x 48, lower) and y as row 48
  __shared__ double yv[48];
  __shared__ int flag;
  const int t = threadIdx.x;
  // Every global load of this prologue (the partial sums, the Gram entries
  // of C and y) is issued before the first one is used: they are L2 misses
  // (written by other workgroups), and one workgroup has nothing else to
  // hide their latency behind.
  const int k1 = d.k1, K = 3 * k1;
  constexpr int kPU = 4;  // partials per thread in the first round (nb <= 1024)
  double pe[kPU][2], pg[kPU][2];
  int pc[kPU][2];
  const int nparts = d.nb + d.nbones;  // element workgroups, then bones
#pragma unroll
  for (int u = 0; u < kPU; ++u) {
    const int b = t + u * kCtlThreads;
    const bool ok = b < nparts;
    pe[u][0] = ok ? d.part_e[2 * b] : 0.0;
    pe[u][1] = ok ? d.part_e[2 * b + 1] : 0.0;
    pg[u][0] = ok ? d.part_g[2 * b] : 0.0;
    pg[u][1] = ok ? d.part_g[2 * b + 1] : 0.0;
    pc[u][0] = ok ? d.part_cnt[2 * b] : 0;
    pc[u][1] = ok ? d.part_cnt[2 * b + 1] : 0;
  }
  // C = Lambda - alpha Gram, lower triangle, padded to 48 x 48 with the
  // identity (unused modes); row r = (c, j) with c = r / k1, j = r % k1
  constexpr int kCU = (48 * 48 + kCtlThreads - 1) / kCtlThreads;
  double g1v[kCU], g2v[kCU], nuv[kCU];
#pragma unroll
  for (int u = 0; u < kCU; ++u) {
    const int idx = t + u * kCtlThreads;
    const int r = idx / 48, q = idx % 48;
    const bool in = idx < 48 * 48 && q <= r && r < K;
    const int c = (r >= k1) + (r >= 2 * k1), j = r - c * k1;
    const int cp = (q >= k1) + (q >= 2 * k1), jp = q - cp * k1;
    // lower triangle: c >= cp; the stored pair is (cp, c)
    const int pair = cp == 0 ? c : (cp == 1 ? 2 + c : 5);
    g1v[u] = in ? d.gram[pair * 256 + jp * 16 + j] : 0.0;
    g2v[u] = in && c == cp ? d.gram[pair * 256 + j * 16 + jp] : 0.0;
    nuv[u] = in && r == q ? d.nu[j] : 0.0;
  }
  const double yload = t < K ? d.gram[1536 + ((t >= k1) + (t >= 2 * k1)) * 16 + (t - ((t >= k1) + (t >= 2 * k1)) * k1)] : 0.0;
  DD acc[2] = {DD{0, 0}, DD{0, 0}};
  int cl = 0, inv = 0;
#pragma unroll
  for (int u = 0; u < kPU; ++u)
    if (t + u * kCtlThreads < nparts) {
      acc[0] = dd_add(acc[0], DD{pe[u][0], pe[u][1]});
      acc[1] = dd_add(acc[1], DD{pg[u][0], pg[u][1]});
      cl += pc[u][0];
      inv += pc[u][1];
    }
  for (int b = t + kPU * kCtlThreads; b < nparts; b += kCtlThreads) {
    acc[0] = dd_add(acc[0], DD{d.part_e[2 * b], d.part_e[2 * b + 1]});
    acc[1] = dd_add(acc[1], DD{d.part_g[2 * b], d.part_g[2 * b + 1]});
    cl += d.part_cnt[2 * b];
    inv += d.part_cnt[2 * b + 1];
  }
#pragma unroll
  for (int u = 0; u < kCU; ++u) {
    const int idx = t + u * kCtlThreads;
    const int r = idx / 48, q = idx % 48;
    if (idx < 48 * 48 && q <= r) {
      double v = (r == q) ? 1.0 : 0.0;
      if (r < K) {
        const int c = (r >= k1) + (r >= 2 * k1);
        const int cp = (q >= k1) + (q >= 2 * k1);
        const double g = c == cp ? 0.5 * (g1v[u] + g2v[u]) : g1v[u];
        v = nuv[u] - d.alpha * g;
      }
      Cm[r][q] = v;
    }
  }
  if (t < 48) Cm[48][t] = yload;
  block_reduce_dd_int2<2, kCtlThreads>(acc, cl, inv, sh, cnt[0]);
  const int cl_sum = cl, inv_sum = inv;
  if (t == 0) {
    const double g2 = acc[1].hi + acc[1].lo;
    ctl->energy = acc[0].hi + acc[0].lo;
    ctl->gnorm2 = g2;
    ctl->clamped = cl_sum;
    ctl->inverted = inv_sum;
    if (ctl->iter == 0 && ctl->gnorm0_2 < 0) ctl->gnorm0_2 = g2;
    int stop = 0;
    if (!(g2 == g2) || !(ctl->energy == ctl->energy) || g2 > 1e300) {
      ctl->status = EMU_E_NONFINITE_CODE;
      stop = 1;
    } else if (!ctl->eval_only && (g2 <= ctl->tol2 || (ctl->rtol2 > 0 && g2 <= ctl->rtol2 * ctl->gnorm0_2))) {
      ctl->status = 0;
      stop = 1;
    } else if (!ctl->eval_only && ctl->iter >= ctl->max_iters) {
      ctl->status = EMU_E_NOT_CONVERGED_CODE;
      stop = 1;
    }
    flag = stop;
    if (stop) ctl->done = 1;
  }
  __syncthreads();
  if (flag || K == 0) return;
  // Blocked Cholesky of the padded 48 x 48 system by the whole workgroup, in
  // panels of six columns (two barriers per panel), with y appended as row
  // 48: the factor of [C y; y^T *] has (L^{-1} y)^T in that row, so the
  // forward substitution comes with the factorization.  Phase A: every thread
  // factors the 6x6 diagonal block (redundantly, from LDS; pivots by one
  // reciprocal square root), thread 0 stores it and thread t below it
  // solves its row of the panel, L[t][jb..jb+5], into LDS.  Phase B: thread
  // t owns the lower-triangle entries e = t + 256 q (kept in registers) and
  // subtracts the panel's rank-6 product from those right of the panel; the
  // entries of the next panel go to LDS.  A non-positive pivot marks the
  // system as failed (z = 0 below).
  constexpr int NB = 6;
  constexpr int kOwn = (49 * 50 / 2 - 1 + kCtlThreads - 1) / kCtlThreads;
  __shared__ double invp[48];
  __shared__ int nbad;
  int er[kOwn], ec[kOwn];
  double ev[kOwn];
#pragma unroll
  for (int q = 0; q < kOwn; ++q) {
    int e = t + q * kCtlThreads;
    if (e >= 49 * 50 / 2 - 1) e = -1;  // every entry of rows 0..48 but (48, 48)
    // row of packed lower-triangle entry e: r (r + 1) / 2 <= e < (r + 1) (r + 2) / 2,
    // from the float root (within one of the exact value for e < 1224) and
    // one correction each way
    int r = e >= 0 ? (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f) : 0;
    r += (r + 1) * (r + 2) / 2 <= e ? 1 : 0;
    r -= r * (r + 1) / 2 > e ? 1 : 0;
    er[q] = e >= 0 ? r : 0;
    ec[q] = e >= 0 ? e - r * (r + 1) / 2 : 48;  // 48: not owned
    ev[q] = e >= 0 ? Cm[er[q]][ec[q]] : 0.0;
  }
  int nbad_local = 0;
  for (int jb = 0; jb < 48; jb += NB) {
    double Lb[NB][NB], rdg[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        double x = Cm[jb + i][jb + j];
#pragma unroll
        for (int k = 0; k < j; ++k) x -= Lb[i][k] * Lb[j][k];
        if (i == j) {
          nbad_local += !(x > 0);
          const double rx = x > 0 ? rsq(x) : 1.0;
          Lb[i][i] = x > 0 ? x * rx : 1.0;
          rdg[i] = rx;
        } else {
          Lb[i][j] = x * rdg[j];
        }
      }
    if (t == 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) Cm[jb + i][jb + j] = Lb[i][j];
        invp[jb + i] = rdg[i];
      }
    }
    if (t >= jb + NB && t < 49) {
      double l[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        double x = Cm[t][jb + k];
#pragma unroll
        for (int m = 0; m < k; ++m) x -= l[m] * Lb[k][m];
        l[k] = x * rdg[k];
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) Cm[t][jb + k] = l[k];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kOwn; ++q) {
      if (ec[q] >= jb + NB && ec[q] < 48) {
        double s = 0;
#pragma unroll
        for (int k = 0; k < NB; ++k) s += Cm[er[q]][jb + k] * Cm[ec[q]][jb + k];
        ev[q] -= s;
        if (ec[q] < jb + 2 * NB) Cm[er[q]][ec[q]] = ev[q];
      }
    }
    __syncthreads();
  }
  if (t == 0) nbad = nbad_local;
  __syncthreads();
  const int bad = nbad > 0;
  for (int idx = t; idx < 48 * 48; idx += kCtlThreads) {
    const int r = idx / 48, c = idx % 48;
    d.cfac[idx] = c <= r ? Cm[r][c] : 0.0;
  }
  if (t >= 64) return;
  // backward substitution L^T z = L^{-1} y in the first wave (the forward one
  // is row 48 of the factor): lane t holds entry t; the newly solved entry is
  // broadcast with readlane.  Lane t's column of L and the pivots are read
  // from LDS ahead of the dependent chain, which then runs on registers only.
  double yt = t < 48 ? Cm[48][t] : 0.0;
  double lv[48], ip[48];
#pragma unroll
  for (int i = 0; i < 48; ++i) {
    lv[i] = t < 48 && i > t ? Cm[i][t] : 0.0;
    ip[i] = invp[i];
  }
#pragma unroll
  for (int i = 47; i >= 0; --i) {
    const double zi = bcast_lane(yt, i) * ip[i];
    yt = t == i ? zi : yt - lv[i] * zi;
  }
  if (t < 48) yv[t] = yt;
  __builtin_amdgcn_wave_barrier();
  if (t == 0 && bad) ctl->chol_fail += 1;
  if (t == 0) d.cfac_ok[0] = !bad;
  if (t < 48) {
    const int c = t / kMaxK1, j = t % kMaxK1;
    d.zbuf[t] = (!bad && j < k1) ? yv[c * k1 + j] : 0.0;
  }
}
__global__ void __launch_bounds__(kCtlThreads) k_control_a(DevMesh d) { b_control_a(d, blockIdx.x); }

// uz[v][c] = sum_j z[(c,j)] phi_j(v)  (zero at pinned vertices).  Four lanes
// per vertex: lane s takes modes 4s .. 4s + 3 (two 16-byte loads, so a wave
// reads 16 consecutive rows of phi), and the four partial sums are added in a
// fixed order, (a0 + a1) + (a2 + a3); lanes s = 0, 1, 2 store coordinate s.
constexpr int kUzLanes = 4;
DEV void b_uz(const DevMesh& d, int bid) {
  const int t = bid * kBlock + threadIdx.x;
  const int v = t / kUzLanes, s = t % kUzLanes;
  if (stopped(d, v < d.n ? d.phi[(int64_t)kMaxK1 * v] : 0.0)) return;
  double a[3] = {0, 0, 0};
  if (v < d.n && d.k1 > 0) {
    const double2* ph = reinterpret_cast<const double2*>(d.phi + (int64_t)kMaxK1 * v + 4 * s);
    const double2 p0 = ph[0], p1 = ph[1];
    const double p[4] = {p0.x, p0.y, p1.x, p1.y};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) a[c] += d.zbuf[c * kMaxK1 + 4 * s + q] * p[q];
  }
#pragma unroll
  for (int off = 1; off < kUzLanes; off <<= 1)
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c] += __shfl_xor(a[c], off);
  if (v >= d.n || s >= 3) return;
  d.uz[3 * v + s] = s == 0 ? a[0] : (s == 1 ? a[1] : a[2]);
}
__global__ void __launch_bounds__(kBlock) k_uz(DevMesh d) { b_uz(d, blockIdx.x); }

// Direction: d = gbar + alpha H^{-1} B^T z with B^T z = w Y^T vec(R^T G uz);
// p = -d; contributions of dF = R D(p).  (The Armijo slope g.p is the exact
// linear coefficient of the line-search polynomial.)
template <typename T, bool kC = false>
DEV void b_direction(const DevMesh& d, int bid) {
  {
    const int i0 = xcd_block(bid, d.nb) * kBlock + threadIdx.x;
    if (stopped(d, i0 < d.m ? d.w[i0] : 0.0)) return;
  }
  const int m = d.m;
  const T* Lf = (const T*)d.Lf;
  const T* gbar = (const T*)d.gbar;
  for (int i = xcd_block(bid, d.nb) * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    if (d.nbones && d.bone_pos[i] >= 0) continue;  // affine bone tets: k_bone_dir
    Elem e;
    load_elem(d, i, e);
    double R[9], Az[9], RA[9];
    load_R(d, i, R);
    gather_grad(d.uz, e, Az);
    matTmul3(R, Az, RA);
    T ty[9];
    to_y<T, double>(RA, ty);
    T Ds[21], Dk[6], gb[9];
#pragma unroll
    for (int k = 0; k < 21; ++k) Ds[k] = Lf[k * m + i];
#pragma unroll
    for (int k = 0; k < 6; ++k) Dk[k] = Lf[(21 + k) * m + i];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      gb[k] = gbar[k * m + i];
      ty[k] *= (T)e.w;
    }
    hinv_apply<T, kC>(d, i, Ds, Dk, ty);
    double p[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      p[k] = -((double)gb[k] + d.alpha * (double)ty[k]);
      d.p[k * m + i] = p[k];
    }
    double D[9], dF[9];
    from_y<double>(p, D);
    matmul3(R, D, dF);
    write_contrib(d, i, e, dF);
  }
}
template <typename T, bool kC = false>
__global__ void __launch_bounds__(kBlock) k_direction(DevMesh d) { b_direction<T, kC>(d, blockIdx.x); }

// ------------------------------------------------------------------ affine bones
// Sec. 3.3: the tets of a bone share one deformation gradient F_b.  Each bone
// tet keeps a copy of F_b = R_b S_b (the accept step applies the same p_b to
// every copy, so the copies stay identical), and the reduced variable's
// quantities are sums over its tets, all in the shared rotated frame:
//   gradient  g_b = sum_i g_i
//   block     H_b = definiteness fix of the blocks of sum_i vol_i d2Psi_i(S_b)
//                   + alpha sum_i w_i I  (d2Psi is linear in vol mu and vol lhat
//                   at a fixed S; bone tets are passive)
//   low rank  B_b = sum_i B_i, i.e. Gamma_b[j] = sum_i w_i gphi_j(i)
// The bone's block inverses and gbar_b sit at its representative tet (its
// first in element order).  The per-element passes leave bone tets out (the
// element pass keeps their gradients aside and out of the norm, the Hessian
// pass writes identity blocks for them, the Gram pass weights them 0, the
// direction pass leaves them to k_bone_dir).  One workgroup per bone, a fixed assignment of its tets to
// threads and fixed-order sums; its partial sums take the slots after the
// element workgroups'.
constexpr int kBoneSums = 9 + 3 * kMaxK1 + 3;  // g, Gamma, vol mu, vol lhat, w

template <int N>
DEV void block_sum_fixed(double (&v)[N], double (*red)[N]) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) red[wave][k] = v[k];
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_bone_blocks(DevMesh d) {
  if (d.ctl->done) return;
  const int b = blockIdx.x, t = threadIdx.x, m = d.m;
  const int p0 = d.bone_ptr[b], p1 = d.bone_ptr[b + 1];
  __shared__ double red[kBlock / 64][kBoneSums];
  __shared__ double tot[kBoneSums];
  __shared__ T zr[kGramRow];
  double acc[kBoneSums];
#pragma unroll
  for (int k = 0; k < kBoneSums; ++k) acc[k] = 0.0;
  for (int q = p0 + t; q < p1; q += kBlock) {
    const int i = d.bone_el[q];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] += d.bone_gbuf[(int64_t)k * d.nbt + q];
    Elem e;
    load_elem(d, i, e);
    for (int j = 0; j < d.k1; ++j) {
      double g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double ph = d.phi[(int64_t)kMaxK1 * e.v[v] + j];
        g0 += ph * e.b[v][0];
        g1 += ph * e.b[v][1];
        g2 += ph * e.b[v][2];
      }
#pragma unroll
      for (int jj = 0; jj < kMaxK1; ++jj)
        if (jj == j) {
          acc[9 + 3 * jj] += e.w * g0;
          acc[9 + 3 * jj + 1] += e.w * g1;
          acc[9 + 3 * jj + 2] += e.w * g2;
        }
    }
    acc[kBoneSums - 3] += e.vol * e.mu;
    acc[kBoneSums - 2] += e.vol * e.lhat;
    acc[kBoneSums - 1] += e.w;
  }
  block_sum_fixed<kBoneSums>(acc, red);
  if (t < kBoneSums) {
    double v = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) v += red[w][t];
    tot[t] = v;
  }
  __syncthreads();
  const int rep = d.bone_el[p0];
  T* Lf = (T*)d.Lf;
  T* gbar = (T*)d.gbar;
  if (t == 0) {
    double S[9];
    load_S(d, rep, S);
    const double u[3] = {0, 0, 1};
    T Hs[6][6], Hk[3][3];
    hess_blocks_s<T>(S, tot[kBoneSums - 3], tot[kBoneSums - 2], 0.0, u, Hs, Hk);
    const T beta = (T)(d.alpha * tot[kBoneSums - 1]);
    T Ls[21], Lk[6], Ds[21], Dk[6];
    const int ncl = clamp_add_factor<T, 6>(Hs, beta, Ls) + clamp_add_factor<T, 3>(Hk, beta, Lk);
    chol_inverse<T, 6>(Ls, Ds);
    chol_inverse<T, 3>(Lk, Dk);
    T gy[9];
    double g2 = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      gy[k] = (T)tot[k];
      g2 += tot[k] * tot[k];
    }
    split_apply<T>(Ds, Dk, gy);
#pragma unroll
    for (int k = 0; k < 21; ++k) Lf[k * m + rep] = Ds[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) Lf[(21 + k) * m + rep] = Dk[k];
#pragma unroll
    for (int k = 0; k < 9; ++k) gbar[k * m + rep] = gy[k];
    const int slot = d.nb + b;
    d.part_e[2 * slot] = 0.0;
    d.part_e[2 * slot + 1] = 0.0;
    d.part_g[2 * slot] = g2;
    d.part_g[2 * slot + 1] = 0.0;
    d.part_cnt[2 * slot] = ncl;
    d.part_cnt[2 * slot + 1] = 0;
  }
  __syncthreads();
  // the bone's Z blocks (three lanes, as in the Gram pass) and R D(gbar_b)
  if (t < 3) {
    gram_zblocks<T, false>(d, rep, t, zr);
    double gbd[9], D[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) gbd[q] = (double)gbar[q * m + rep];
    from_y<double>(gbd, D);
    const double r0 = d.R[(3 * t) * m + rep], r1 = d.R[(3 * t + 1) * m + rep], r2 = d.R[(3 * t + 2) * m + rep];
#pragma unroll
    for (int q = 0; q < 3; ++q) zr[54 + 3 * t + q] = (T)(r0 * D[q] + r1 * D[3 + q] + r2 * D[6 + q]);
  }
  __syncthreads();
  // its Gram row: [p][x][y] = Gamma_x^T Z_p Gamma_y, and y[(c, j)] = Gamma_j . (R D(gbar))_c
  double* out = d.part_gram + (int64_t)(d.nbg + b) * kGramEntries;
  for (int e = t; e < kGramEntries; e += kBlock) {
    double v = 0;
    if (e < 1536) {
      const int pp = e >> 8, x = (e >> 4) & 15, y = e & 15;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) v += tot[9 + 3 * x + a] * (double)zr[pp * 9 + a * 3 + c] * tot[9 + 3 * y + c];
    } else {
      const int c = (e - 1536) >> 4, j = (e - 1536) & 15;
#pragma unroll
      for (int a = 0; a < 3; ++a) v += tot[9 + 3 * j + a] * (double)zr[54 + 3 * c + a];
    }
    out[e] = v;
  }
}

// The bone's step p_b = -(gbar_b + alpha H_b^{-1} R_b^T sum_i w_i A_z(i)) (A_z:
// the compatible gradient of Phi^T z at tet i), copied to every bone tet with
// its ACAP right-hand-side contribution.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bone_dir(DevMesh d) {
  if (d.ctl->done) return;
  const int b = blockIdx.x, t = threadIdx.x, m = d.m;
  const int p0 = d.bone_ptr[b], p1 = d.bone_ptr[b + 1];
  __shared__ double red[kBlock / 64][9];
  __shared__ double pb[9];
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int q = p0 + t; q < p1; q += kBlock) {
    const int i = d.bone_el[q];
    Elem e;
    load_elem(d, i, e);
    double Az[9];
    gather_grad(d.uz, e, Az);
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] += e.w * Az[k];
  }
  block_sum_fixed<9>(acc, red);
  const int rep = d.bone_el[p0];
  if (t == 0) {
    double u[9], R[9], RA[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    load_R(d, rep, R);
    matTmul3(R, u, RA);
    const T* Lf = (const T*)d.Lf;
    const T* gbar = (const T*)d.gbar;
    T Ds[21], Dk[6], ty[9];
#pragma unroll
    for (int k = 0; k < 21; ++k) Ds[k] = Lf[k * m + rep];
#pragma unroll
    for (int k = 0; k < 6; ++k) Dk[k] = Lf[(21 + k) * m + rep];
    to_y<T, double>(RA, ty);
    split_apply<T>(Ds, Dk, ty);
#pragma unroll
    for (int k = 0; k < 9; ++k) pb[k] = -((double)gbar[k * m + rep] + d.alpha * (double)ty[k]);
  }
  __syncthreads();
  double D[9], R[9], dF[9];
  from_y<double>(pb, D);
  load_R(d, rep, R);
  matmul3(R, D, dF);
  for (int q = p0 + t; q < p1; q += kBlock) {
    const int i = d.bone_el[q];
#pragma unroll
    for (int k = 0; k < 9; ++k) d.p[k * m + i] = pb[k];
    Elem e;
    load_elem(d, i, e);
    write_contrib(d, i, e, dF);
  }
}

// Line-search polynomial: E(sigma) - E(0) = sum_k c_k sigma^k (k = 1..6), exact
// per element along F(sigma) = R (S + sigma D), A(sigma) = A + sigma dA.
DEV void b_lscoef(const DevMesh& d, int bid) {
  {
    const int i0 = xcd_block(bid, d.nb) * kBlock + threadIdx.x;
    if (stopped(d, i0 < d.m ? d.vol[i0] : 0.0)) return;
  }
  __shared__ DD sh[6 * kBlock];
  DD acc[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) acc[k] = DD{0, 0};
  const int m = d.m;
  for (int i = xcd_block(bid, d.nb) * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    Elem e;
    load_elem(d, i, e);
    double R[9], S[9], py[9], D[9], A[9], dA[9], At[9], dAt[9];
    load_R(d, i, R);
    load_S(d, i, S);
#pragma unroll
    for (int k = 0; k < 9; ++k) py[k] = d.p[k * m + i];
    from_y<double>(py, D);
    gather_grad(d.q, e, A);
    gather_grad(d.dq, e, dA);
    matTmul3(R, A, At);
    matTmul3(R, dA, dAt);
    const double J = det3(S);
    double CS[9], CD[9];
    cof3<double>(S, CS);
    cof3<double>(D, CD);
    double j1 = 0, j2 = 0, sd = 0, dd2 = 0, r1 = 0, r2 = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      j1 += CS[k] * D[k];
      j2 += S[k] * CD[k];
      sd += S[k] * D[k];
      dd2 += D[k] * D[k];
      const double res = At[k] - S[k], dres = dAt[k] - D[k];
      r1 += res * dres;
      r2 += dres * dres;
    }
    const double j3 = det3(D);
    double Su[3], Du[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Su[c] = S[3 * c] * e.u[0] + S[3 * c + 1] * e.u[1] + S[3 * c + 2] * e.u[2];
      Du[c] = D[3 * c] * e.u[0] + D[3 * c + 1] * e.u[1] + D[3 * c + 2] * e.u[2];
    }
    const double f1 = Su[0] * Du[0] + Su[1] * Du[1] + Su[2] * Du[2];
    const double f2 = Du[0] * Du[0] + Du[1] * Du[1] + Du[2] * Du[2];
    const double mu = e.mu, lh = e.lhat, Jm = J - 1.0, afk = e.a * d.kf, beta = d.alpha * e.w;
    double c[6];
    c[0] = mu * sd - mu * j1 + lh * Jm * j1 + 2.0 * afk * f1;
    c[1] = 0.5 * mu * dd2 - mu * j2 + lh * Jm * j2 + 0.5 * lh * j1 * j1 + afk * f2;
    c[2] = -mu * j3 + lh * Jm * j3 + lh * j1 * j2;
    c[3] = 0.5 * lh * (j2 * j2 + 2.0 * j1 * j3);
    c[4] = lh * j2 * j3;
    c[5] = 0.5 * lh * j3 * j3;
#pragma unroll
    for (int k = 0; k < 6; ++k) c[k] *= e.vol;
    c[0] += beta * r1;
    c[1] += 0.5 * beta * r2;
    if (d.has_ext) {
      // change of the external work along the step: nu . dF = (R^T nu) . D
      double nu[9], nur[9];
      gather_grad(d.vext, e, nu);
      matTmul3(R, nu, nur);
      double wd = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) wd += nur[k] * D[k];
      c[0] -= e.w * wd;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = dd_add_d(acc[k], c[k]);
  }
  block_reduce_dd<6>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      d.part_ls[2 * kLsTerms * bid + 2 * k] = acc[k].hi;
      d.part_ls[2 * kLsTerms * bid + 2 * k + 1] = acc[k].lo;
    }
}
__global__ void __launch_bounds__(kBlock) k_lscoef(DevMesh d) { b_lscoef(d, blockIdx.x); }

// Single workgroup: Armijo backtracking on the exact polynomial (Algorithm 1).
DEV void b_control_b(const DevMesh& d, int bid) {
  Ctl* ctl = d.ctl;
  const int t = threadIdx.x;
  if (stopped(d, t < d.nb ? d.part_ls[2 * kLsTerms * t] : 0.0)) return;
  __shared__ DD sh[kLsTerms * kBlock];
  DD acc[kLsTerms];
#pragma unroll
  for (int k = 0; k < kLsTerms; ++k) acc[k] = DD{0, 0};
  for (int b = t; b < d.nb; b += kBlock)
#pragma unroll
    for (int k = 0; k < kLsTerms; ++k)
      acc[k] = dd_add(acc[k], DD{d.part_ls[2 * kLsTerms * b + 2 * k], d.part_ls[2 * kLsTerms * b + 2 * k + 1]});
  block_reduce_dd<kLsTerms>(acc, sh);
  if (t != 0) return;
  double c[6];
  for (int k = 0; k < 6; ++k) c[k] = acc[k].hi + acc[k].lo;
  // Slope of the Armijo test: the directional derivative g . p = dE/dsigma at
  // 0, which is the linear coefficient c[0] of the energy polynomial (the
  // ACAP term's change through q cancels at q*).  It is an FP64 double-double
  // sum in both precisions, so the decision stays FP64 (form (1)).
  const double gtp = c[0];
  ctl->gtp = gtp;
  ctl->solves += 1;
  const double g2 = ctl->gnorm2, g02 = ctl->gnorm0_2;
  const bool stalled = ctl->stall_rel > 0 && g2 <= ctl->stall_rel * ctl->stall_rel * g02;
  if (!(gtp < 0.0)) {
    // no descent direction: at the rounding floor of the gradient this is
    // convergence (mixed path, |g| <= stall_rel |g_0|), otherwise a failure
    ctl->status = stalled ? 0 : EMU_E_LINESEARCH_CODE;
    ctl->sigma = 0.0;
    ctl->done = 1;
    return;
  }
  double sg = ctl->sigma0;
  int ok = 0, tr = 0;
  for (int j = 0; j <= 40; ++j) {
    ++tr;
    const double dE = sg * (c[0] + sg * (c[1] + sg * (c[2] + sg * (c[3] + sg * (c[4] + sg * c[5])))));
    if (dE <= ctl->armijo_c * sg * gtp) {
      ok = 1;
      break;
    }
    sg *= ctl->rho;
  }
  ctl->trials += tr;
  if (ok) {
    ctl->sigma = sg;
    ctl->iter += 1;
  } else {
    ctl->sigma = 0.0;
    ctl->status = stalled ? 0 : EMU_E_LINESEARCH_CODE;
    ctl->done = 1;
  }
}
__global__ void __launch_bounds__(kBlock) k_control_b(DevMesh d) { b_control_b(d, blockIdx.x); }

// ------------------------------------------------------------------ adjoint
// Exact Hessian-vector products and the quasi-Newton preconditioner used by
// the adjoint conjugate-gradient solve.  Vectors over elements are F-coordinate
// fields in world frame, structure of arrays [9][m].

// per-thread sum of 2 values into a block partial (double-double)
template <int NV>
DEV void write_partial(DD (&acc)[NV], DD* sh, double* out) {
  block_reduce_dd<NV>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      out[2 * k] = acc[k].hi;
      out[2 * k + 1] = acc[k].lo;
    }
}

// ACAP right-hand-side contributions of a field V ([9][m])
__global__ void __launch_bounds__(kBlock) k_contrib_field(DevMesh d, const double* V, int check_done) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m || (check_done && d.ctl->done)) return;
  Elem e;
  load_elem(d, i, e);
  double F[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) F[k] = V[k * d.m + i];
  write_contrib(d, i, e, F);
}

// b_i = w_i A_i(x)  (x: vertex field [n][3], zero at pins)
__global__ void __launch_bounds__(kBlock) k_weighted_grad(DevMesh d, const double* x, double* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  Elem e;
  load_elem(d, i, e);
  double A[9];
  gather_grad(x, e, A);
#pragma unroll
  for (int k = 0; k < 9; ++k) out[k * d.m + i] = e.w * A[k];
}

// ------------------------------------------------------------------ device eigenpairs
// The lowest eigenpairs of L_ff (the modes of eq. low-rank) by block inverse
// subspace iteration with the device factor.  A block is kEigCols columns in
// kEigCols / 3 packs; a pack is a vertex field in the sweeps' [n][3] layout
// (column 3 p + c of the block is component c of pack p, free rows first,
// pinned rows zero); packs are pstride doubles apart.

// V = G x per element (unweighted): L x = G^T W G x through the ACAP
// right-hand side of V.
__global__ void __launch_bounds__(kBlock) k_grad_field(DevMesh d, const double* x, double* V) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  Elem e;
  load_elem(d, i, e);
  double A[9];
  gather_grad(x, e, A);
#pragma unroll
  for (int k = 0; k < 9; ++k) V[k * d.m + i] = A[k];
}

DEV double eig_at(const double* A, int64_t pstride, int row, int col) {
  return A[(col / 3) * pstride + 3 * (int64_t)row + (col % 3)];
}

// Partial products A^T B (kEigCols x kEigCols) of a contiguous row range per
// workgroup, in tiles of kEigTile rows staged in LDS; part[blk][a * kEigCols + b].
constexpr int kEigTile = 32;
constexpr int kEigPairs = kEigCols * kEigCols;
constexpr int kEigPerThread = (kEigPairs + kBlock - 1) / kBlock;
__global__ void __launch_bounds__(kBlock) k_eig_gram(int nf, int64_t pstride, const double* A, const double* B,
                                                     int rows_per_blk, double* part) {
  __shared__ double ta[kEigTile][kEigCols], tb[kEigTile][kEigCols];
  const int t = threadIdx.x;
  const int r0 = blockIdx.x * rows_per_blk, r1 = min(nf, r0 + rows_per_blk);
  double acc[kEigPerThread];
#pragma unroll
  for (int q = 0; q < kEigPerThread; ++q) acc[q] = 0.0;
  for (int base = r0; base < r1; base += kEigTile) {
    const int nr = min(kEigTile, r1 - base);
    __syncthreads();
    for (int k = t; k < kEigTile * kEigCols; k += kBlock) {
      const int rr = k / kEigCols, c = k % kEigCols;
      ta[rr][c] = rr < nr ? eig_at(A, pstride, base + rr, c) : 0.0;
      tb[rr][c] = rr < nr ? eig_at(B, pstride, base + rr, c) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kEigPerThread; ++q) {
      const int pr = t + q * kBlock;
      if (pr < kEigPairs) {
        const int a = pr / kEigCols, b = pr % kEigCols;
        double s = acc[q];
        for (int rr = 0; rr < kEigTile; ++rr) s += ta[rr][a] * tb[rr][b];
        acc[q] = s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kEigPerThread; ++q) {
    const int pr = t + q * kBlock;
    if (pr < kEigPairs) part[(int64_t)blockIdx.x * kEigPairs + pr] = acc[q];
  }
}
// out[e] = sum over blocks of part[blk][e], in block order
__global__ void __launch_bounds__(kBlock) k_eig_reduce(int nblk, int nent, const double* part, double* out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= nent) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * nent + e];
  out[e] = s;
}
// X = Y W (W kEigCols x kEigCols, row-major), one row per thread
__global__ void __launch_bounds__(kBlock) k_eig_mul(int nf, int64_t pstride, const double* Y, const double* W,
                                                    double* X) {
  __shared__ double w[kEigPairs];
  for (int k = threadIdx.x; k < kEigPairs; k += kBlock) w[k] = W[k];
  __syncthreads();
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nf) return;
  double y[kEigCols];
#pragma unroll
  for (int c = 0; c < kEigCols; ++c) y[c] = eig_at(Y, pstride, i, c);
  for (int j = 0; j < kEigCols; ++j) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kEigCols; ++c) s += y[c] * w[c * kEigCols + j];
    X[(j / 3) * pstride + 3 * (int64_t)i + (j % 3)] = s;
  }
}
// part[blk][j] = sum over the block's rows of (LX[:, j] - lam[j] X[:, j])^2, j < ncols
__global__ void __launch_bounds__(kBlock) k_eig_resid(int nf, int64_t pstride, const double* X, const double* LX,
                                                      const double* lam, int ncols, double* part) {
  __shared__ double red[kBlock / 64][kEigCols];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < ncols; ++j) {
    double r = 0.0;
    if (i < nf) {
      const double dv = eig_at(LX, pstride, i, j) - lam[j] * eig_at(X, pstride, i, j);
      r = dv * dv;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off);
    if (lane == 0) red[wave][j] = r;
  }
  __syncthreads();
  if (threadIdx.x < ncols) {
    const int j = threadIdx.x;
    part[(int64_t)blockIdx.x * ncols + j] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
  }
}

// ------------------------------------------------------------------ contact
// Algorithm 1's contact loop (Sec. 3.5) against analytic obstacles: rows
// (n, b) of half-spaces (a vertex x with n . x < b penetrates by b - n . x and
// is pushed along n), then rows (c, r) of spheres (|x - c| < r: depth
// r - |x - c|, pushed along (x - c) / |x - c|).  Penalty force k * depth per
// free vertex, written to d.rhs (the right-hand side of the sweeps); block
// partials of |f|^2, added in a fixed order.
__global__ void __launch_bounds__(kBlock) k_contact_force(DevMesh d, const double* obs, int np, int ns, double k,
                                                          double* part) {
  __shared__ double red[kBlock / 64];
  const int v = blockIdx.x * kBlock + threadIdx.x;
  double f0 = 0, f1 = 0, f2 = 0;
  if (v < d.nf) {
    const double x0 = d.q[3 * v], x1 = d.q[3 * v + 1], x2 = d.q[3 * v + 2];
    for (int o = 0; o < np; ++o) {
      const double* P = obs + 4 * o;
      const double dep = P[3] - (P[0] * x0 + P[1] * x1 + P[2] * x2);
      if (dep > 0.0) {
        f0 += k * dep * P[0];
        f1 += k * dep * P[1];
        f2 += k * dep * P[2];
      }
    }
    for (int o = np; o < np + ns; ++o) {
      const double* Q = obs + 4 * o;
      const double r0 = x0 - Q[0], r1 = x1 - Q[1], r2 = x2 - Q[2];
      const double dist = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
      if (dist < Q[3] && dist > 0.0) {
        const double sc = k * (Q[3] - dist) / dist;
        f0 += sc * r0;
        f1 += sc * r1;
        f2 += sc * r2;
      }
    }
    d.rhs[3 * v] = f0;
    d.rhs[3 * v + 1] = f1;
    d.rhs[3 * v + 2] = f2;
  }
  double s2 = f0 * f0 + f1 * f1 + f2 * f2;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
// q += x2 at the free vertices (the ACAP response of a contact step z), zc += z
__global__ void __launch_bounds__(kBlock) k_contact_accum(DevMesh d, const double* x2, const double* z, double* zc) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < 3 * (int64_t)d.nf) d.q[t] += x2[t];
  if (t < 9 * (int64_t)d.m) zc[t] += z[t];
}
// The pending step of the iteration together with the contact field zc:
// F <- R (S + sigma D(p)) + zc, re-split; then no step is pending.
__global__ void __launch_bounds__(kBlock) k_accept_contact(DevMesh d, const double* zc) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d.m) return;
  double R[9], S[9];
  load_R(d, i, R);
  load_S(d, i, S);
  accept_elem<true>(d, i, d.ctl->sigma, zc, R, S);
}
__global__ void k_clear_step(DevMesh d) {
  if (threadIdx.x == 0) d.ctl->sigma = 0.0;
}

// out = H v with H = d2E/dF2 = blockdiag(vol d2Psi(F_i)) + alpha W - alpha W G L^{-1} G^T W:
//   out_i = vol d2Psi(F_i)[v_i] + beta_i (v_i - A_i(x)),  x = L^{-1} G^T W v.
// d2Psi[V] in the rotated frame at the symmetric S (X = R^T V):
//   mu X + lhat <cof S, X> cof S + kappa dcof(S)[X] + 2 a kf (X u) u^T,
// with dcof(S)[X] = cof(S + X) - cof(S) - cof(X).  Block partial of v . out.
__global__ void __launch_bounds__(kBlock) k_hvp(DevMesh d, const double* V, const double* x, double* out,
                                                double* part) {
  if (d.ctl->done) return;
  __shared__ DD sh[kBlock];
  DD acc[1] = {DD{0, 0}};
  const int m = d.m;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    Elem e;
    load_elem(d, i, e);
    double R[9], S[9], v[9], X[9], A[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = V[k * m + i];
    load_R(d, i, R);
    load_S(d, i, S);
    matTmul3(R, v, X);
    const double J = det3(S);
    double CS[9], SX[9], CSX[9], CX[9];
    cof3<double>(S, CS);
#pragma unroll
    for (int k = 0; k < 9; ++k) SX[k] = S[k] + X[k];
    cof3<double>(SX, CSX);
    cof3<double>(X, CX);
    double cx = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) cx += CS[k] * X[k];
    const double kap = e.lhat * (J - 1.0) - e.mu, afk2 = 2.0 * e.a * d.kf;
    double Xu[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) Xu[c] = X[3 * c] * e.u[0] + X[3 * c + 1] * e.u[1] + X[3 * c + 2] * e.u[2];
    double HX[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int k = 3 * a + b;
        HX[k] = e.vol * (e.mu * X[k] + e.lhat * cx * CS[k] + kap * (CSX[k] - CS[k] - CX[k]) + afk2 * Xu[a] * e.u[b]);
      }
    double Hv[9];
    matmul3(R, HX, Hv);
    gather_grad(x, e, A);
    const double beta = d.alpha * e.w;
    double vh = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double o = Hv[k] + beta * (v[k] - A[k]);
      out[k * m + i] = o;
      vh += v[k] * o;
    }
    acc[0] = dd_add_d(acc[0], vh);
  }
  write_partial<1>(acc, sh, part + 2 * blockIdx.x);
}

// lam += alpha p, r -= alpha Hp (alpha from the control block); block
// partial of |r|^2
__global__ void __launch_bounds__(kBlock) k_cg_update(DevMesh d, const double* P, const double* HP, double* lam,
                                                      double* r, double* part) {
  if (d.ctl->done) return;
  const double alpha = d.ctl->cg_alpha;
  __shared__ DD sh[kBlock];
  DD acc[1] = {DD{0, 0}};
  const int64_t n9 = 9 * (int64_t)d.m;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n9; k += (int64_t)d.nb * kBlock) {
    lam[k] += alpha * P[k];
    const double rv = r[k] - alpha * HP[k];
    r[k] = rv;
    acc[0] = dd_add_d(acc[0], rv * rv);
  }
  write_partial<1>(acc, sh, part + 2 * blockIdx.x);
}

// p = z + beta p (beta from the control block)
__global__ void __launch_bounds__(kBlock) k_cg_dir(DevMesh d, const double* Z, double* P) {
  if (d.ctl->done) return;
  const double beta = d.ctl->cg_beta;
  const int64_t n9 = 9 * (int64_t)d.m;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n9; k += (int64_t)d.nb * kBlock)
    P[k] = Z[k] + beta * P[k];
}

// Conjugate-gradient scalars of the adjoint, on the device so that the steps
// run without host round trips.  One workgroup: s = the fixed-order
// double-double sum of the nb block partials, then
//   kCgInitRz  rz = s (r . z of the first residual)
//   kCgInitR   |b| = sqrt(s), tol = 1e-10 |b|; stop at once if |b| <= tol,
//              with EMU_E_NONFINITE if |b| is not finite
//   kCgAlpha   alpha = rz / s with s = p . Hp; stop with EMU_E_NONFINITE unless
//              0 < s < inf
//   kCgResid   |r| = sqrt(s) after the update, one more step; stop at
//              |r| <= tol, with EMU_E_NONFINITE if |r| is not finite, or with
//              EMU_E_NOT_CONVERGED at the step cap
//   kCgBeta    beta = s / rz, rz = s (s = r . z of the new residual)
__global__ void __launch_bounds__(kBlock) k_cg_scalar(DevMesh d, const double* part, int what) {
  Ctl* ctl = d.ctl;
  if (ctl->done) return;
  __shared__ DD sh[kBlock];
  DD acc[1] = {DD{0, 0}};
  for (int b = threadIdx.x; b < d.nb; b += kBlock) acc[0] = dd_add(acc[0], DD{part[2 * b], part[2 * b + 1]});
  block_reduce_dd<1>(acc, sh);
  if (threadIdx.x != 0) return;
  const double s = acc[0].hi + acc[0].lo;
  if (what == kCgInitRz) {
    ctl->cg_rz = s;
  } else if (what == kCgInitR) {
    // (fmax would turn a NaN sum into 0, a false convergence)
    const double b = isfinite(s) ? sqrt(fmax(0.0, s)) : s;
    ctl->cg_bnorm = b;
    ctl->cg_rnorm = b;
    ctl->cg_tol = 1e-10 * b;
    if (!isfinite(b)) {
      ctl->status = EMU_E_NONFINITE_CODE;
      ctl->done = 1;
    } else if (!(b > ctl->cg_tol)) {
      ctl->done = 1;
    }
  } else if (what == kCgAlpha) {
    if (!(s > 0.0) || !isfinite(s)) {
      ctl->status = EMU_E_NONFINITE_CODE;
      ctl->done = 1;
    } else {
      ctl->cg_alpha = ctl->cg_rz / s;
    }
  } else if (what == kCgResid) {
    const double r = isfinite(s) ? sqrt(fmax(0.0, s)) : s;
    ctl->cg_rnorm = r;
    ctl->cg_it += 1;
    if (!isfinite(r)) {
      ctl->status = EMU_E_NONFINITE_CODE;
      ctl->done = 1;
    } else if (!(r > ctl->cg_tol)) {
      ctl->done = 1;
    } else if (ctl->cg_it >= ctl->cg_max) {
      ctl->status = EMU_E_NOT_CONVERGED_CODE;
      ctl->done = 1;
    }
  } else {
    ctl->cg_beta = s / ctl->cg_rz;
    ctl->cg_rz = s;
  }
}
// Start of the adjoint's conjugate gradients: clear the stop flag and status
// the element pass may have left, zero alpha (the first update only measures
// |b|), no steps yet, cap max_steps.
__global__ void k_cg_begin(DevMesh d, int max_steps) {
  Ctl* ctl = d.ctl;
  ctl->done = 0;
  ctl->status = 0;
  ctl->cg_alpha = 0.0;
  ctl->cg_beta = 0.0;
  ctl->cg_it = 0;
  ctl->cg_max = max_steps;
}

// Preconditioner, part 1: rbar = H^{-1} Y^T vec(R^T r) (blocks), stored in rbar
// ([9][m]), and block partials of y[(c,j)] = sum_i w_i (R D(rbar) gphi_j)[c].
template <typename T, bool kC = false>
__global__ void __launch_bounds__(kBlock) k_pc1(DevMesh d, const double* r, double* ypart, double* rbar,
                                                int check_done) {
  if (check_done && d.ctl->done) return;
  __shared__ double red[kBlock / 64][48];
  const int m = d.m;
  const T* Lf = (const T*)d.Lf;
  double y[48];
#pragma unroll
  for (int k = 0; k < 48; ++k) y[k] = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    Elem e;
    load_elem(d, i, e);
    double R[9], rv[9], X[9];
    load_R(d, i, R);
#pragma unroll
    for (int k = 0; k < 9; ++k) rv[k] = r[k * m + i];
    matTmul3(R, rv, X);
    T ry[9];
    to_y<T, double>(X, ry);
    T Ls[21], Lk[6];
#pragma unroll
    for (int k = 0; k < 21; ++k) Ls[k] = Lf[k * m + i];
#pragma unroll
    for (int k = 0; k < 6; ++k) Lk[k] = Lf[(21 + k) * m + i];
    hinv_apply<T, kC>(d, i, Ls, Lk, ry);
    double rb[9], D[9], RD[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      rb[k] = (double)ry[k];
      rbar[k * m + i] = rb[k];
    }
    from_y<double>(rb, D);
    matmul3(R, D, RD);
    // mode gradients gphi_j = sum_v phi_j(v) b_v, four modes of the four
    // vertices per round (16-byte loads of the vertex rows); the mode index
    // is a compile-time constant, so y stays in registers
#pragma unroll
    for (int q4 = 0; q4 < kMaxK1; q4 += 4) {
      double ph[4][4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double2* pr = reinterpret_cast<const double2*>(d.phi + (int64_t)kMaxK1 * e.v[v] + q4);
        const double2 p0 = pr[0], p1 = pr[1];
        ph[v][0] = p0.x;
        ph[v][1] = p0.y;
        ph[v][2] = p1.x;
        ph[v][3] = p1.y;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q4 + q >= d.k1) break;  // uniform
        double g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          g0 += ph[v][q] * e.b[v][0];
          g1 += ph[v][q] * e.b[v][1];
          g2 += ph[v][q] * e.b[v][2];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
          y[c * kMaxK1 + q4 + q] += e.w * (RD[3 * c] * g0 + RD[3 * c + 1] * g1 + RD[3 * c + 2] * g2);
      }
    }
  }
  // wave butterfly, then the 4 waves in order
#pragma unroll
  for (int k = 0; k < 48; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) y[k] += __shfl_xor(y[k], off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 48; ++k) red[wave][k] = y[k];
  __syncthreads();
  if (threadIdx.x < 48) {
    double s0 = 0;
#pragma unroll
    for (int w2 = 0; w2 < kBlock / 64; ++w2) s0 += red[w2][threadIdx.x];
    ypart[48 * blockIdx.x + threadIdx.x] = s0;
  }
}

// Preconditioner, part 2 (one workgroup of kPcThreads): y = sum of partials,
// z = C^{-1} y with the Cholesky factor of C kept by the last element/Gram
// pass.  Wave g adds the partials of workgroups g, g + W, ... (four loads in
// flight) while the workgroup stages the factor in LDS; the W wave sums are
// added in order, then wave 0 runs the two substitutions from LDS.
constexpr int kPcThreads = 1024;
__global__ void __launch_bounds__(kPcThreads) k_pc_solve(DevMesh d, const double* ypart, int check_done) {
  if (check_done && d.ctl->done) return;
  constexpr int W = kPcThreads / 64;
  __shared__ double wsum[W][48];
  __shared__ double Lsh[48 * 48];
  __shared__ double yv[48];
  const int t = threadIdx.x, q = t & 63, g = t >> 6;
  const int k1 = d.k1, K = 3 * k1;
  if (q < 48) {
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int b = g;
    for (; b + 3 * W < d.nb; b += 4 * W) {
      s0 += ypart[48 * b + q];
      s1 += ypart[48 * (b + W) + q];
      s2 += ypart[48 * (b + 2 * W) + q];
      s3 += ypart[48 * (b + 3 * W) + q];
    }
    for (; b < d.nb; b += W) s0 += ypart[48 * b + q];
    wsum[g][q] = (s0 + s1) + (s2 + s3);
  }
  for (int k = t; k < 48 * 48; k += kPcThreads) Lsh[k] = d.cfac[k];
  __syncthreads();
  if (t < 48) {
    double s = wsum[0][t];
#pragma unroll
    for (int w = 1; w < W; ++w) s += wsum[w][t];
    yv[t] = s;
  }
  __syncthreads();
  if (K == 0) {
    if (t < 48) d.zbuf[t] = 0.0;
    return;
  }
  if (g != 0) return;
  // wave 0 alone from here: its lanes run in lockstep, so every read of yv
  // below precedes the writes after the substitutions.  Lane t holds entry t
  // (compact index c*k1+j); step i takes entry i from lane i with a lane read
  // (no LDS round trip on the dependent chain) and scales it by 1 / L_ii.
  double yt = 0.0;
  if (t < K) yt = yv[(t / k1) * kMaxK1 + (t % k1)];
  const double rd = t < K ? 1.0 / Lsh[t * 49] : 0.0;
  for (int i = 0; i < K; ++i) {
    const double ui = bcast_lane(yt, i) * bcast_lane(rd, i);
    if (t == i) yt = ui;
    else if (t > i && t < K) yt -= Lsh[t * 48 + i] * ui;
  }
  for (int i = K - 1; i >= 0; --i) {
    const double zi = bcast_lane(yt, i) * bcast_lane(rd, i);
    if (t == i) yt = zi;
    else if (t < i) yt -= Lsh[i * 48 + t] * zi;
  }
  if (t < K) yv[t] = yt;
  wave_sync_mem();
  if (t < 48) {
    const int c = t / kMaxK1, j = t % kMaxK1;
    d.zbuf[t] = (j < k1 && d.cfac_ok[0]) ? yv[c * k1 + j] : 0.0;
  }
}

// Preconditioner, part 3: z_i = R D(rbar_i + alpha H^{-1} w Y^T vec(R^T A_i(uz)))
// (F coordinates); block partials of r . z.
template <typename T, bool kC = false>
__global__ void __launch_bounds__(kBlock) k_pc2(DevMesh d, const double* r, double* zout, double* part,
                                                const double* rbar, int check_done) {
  if (check_done && d.ctl->done) return;
  __shared__ DD sh[kBlock];
  DD acc[1] = {DD{0, 0}};
  const int m = d.m;
  const T* Lf = (const T*)d.Lf;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    Elem e;
    load_elem(d, i, e);
    double R[9], Az[9], RA[9];
    load_R(d, i, R);
    gather_grad(d.uz, e, Az);
    matTmul3(R, Az, RA);
    T ty[9];
    to_y<T, double>(RA, ty);
    T Ls[21], Lk[6];
#pragma unroll
    for (int k = 0; k < 21; ++k) Ls[k] = Lf[k * m + i];
#pragma unroll
    for (int k = 0; k < 6; ++k) Lk[k] = Lf[(21 + k) * m + i];
#pragma unroll
    for (int k = 0; k < 9; ++k) ty[k] *= (T)e.w;
    hinv_apply<T, kC>(d, i, Ls, Lk, ty);
    double zy[9], D[9], Z[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) zy[k] = rbar[k * m + i] + d.alpha * (double)ty[k];
    from_y<double>(zy, D);
    matmul3(R, D, Z);
    double rz = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      zout[k * m + i] = Z[k];
      rz += r[k * m + i] * Z[k];
    }
    acc[0] = dd_add_d(acc[0], rz);
  }
  write_partial<1>(acc, sh, part + 2 * blockIdx.x);
}

// dL/da partials: per group g, sum over its tets of vol (lam_i u).(F_i u)
__global__ void __launch_bounds__(kBlock) k_adj_da(DevMesh d, const double* lam, double* part) {
  const int m = d.m;
  const int ng = d.ngroups;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    const int g = d.grp[i];
    double val = 0.0;
    if (g >= 0) {
      Elem e;
      load_elem(d, i, e);
      double R[9], S[9], F[9], L[9];
      load_R(d, i, R);
      load_S(d, i, S);
      matmul3(R, S, F);
#pragma unroll
      for (int k = 0; k < 9; ++k) L[k] = lam[k * m + i];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double lu = L[3 * c] * e.u[0] + L[3 * c + 1] * e.u[1] + L[3 * c + 2] * e.u[2];
        const double fu = F[3 * c] * e.u[0] + F[3 * c + 1] * e.u[1] + F[3 * c + 2] * e.u[2];
        val += lu * fu;
      }
      val *= e.vol;
    }
    part[i] = val;  // per element; summed per group by k_group_sum
    (void)ng;
  }
}

// dL/da_g = scale * sum over the tets of group g of per[i]: one workgroup per
// group, each thread a fixed strided set of elements in double-double, the
// wave and workgroup sums in a fixed order (deterministic).
__global__ void __launch_bounds__(kBlock) k_group_sum(DevMesh d, const double* per, double scale, double* out) {
  const int g = blockIdx.x;
  __shared__ DD sh[kBlock];
  DD acc[1] = {DD{0, 0}};
  for (int i = threadIdx.x; i < d.m; i += kBlock)
    if (d.grp[i] == g) acc[0] = dd_add_d(acc[0], per[i]);
  block_reduce_dd<1>(acc, sh);
  if (threadIdx.x == 0) out[g] = scale * (acc[0].hi + acc[0].lo);
}

__global__ void __launch_bounds__(kBlock) k_scale_free(DevMesh d, const double* in, double* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * d.nf) return;
  out[i] = in[i];
}

// ------------------------------------------------------------------ launch helpers
// ------------------------------------------------------- batched iteration
// One launch per kernel class covers every mesh of a batch: block b runs block
// map[b].y of mesh map[b].x, with exactly the code and the per-mesh block
// partition of the single-mesh launch, so each mesh's arithmetic (and every
// fixed-order reduction) is the same alone or batched.
#define EMU_BATCHED(NAME, LB, CALL)                                                            \
  __global__ void __launch_bounds__(LB) NAME(const DevMesh* __restrict__ ms,                   \
                                             const int2* __restrict__ map) {                   \
    const int2 e = map[blockIdx.x];                                                            \
    const DevMesh d = ms[e.x];                                                                 \
    CALL;                                                                                      \
  }
EMU_BATCHED(kb_element64, kBlock, b_element<double>(d, e.y))
EMU_BATCHED(kb_element32, kBlock, b_element<float>(d, e.y))
// the Hessian pass with the occupancy bounds of k_element_hess
template <typename T>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8)))
kb_element_hess(const DevMesh* __restrict__ ms, const int2* __restrict__ map) {
  const int2 e = map[blockIdx.x];
  const DevMesh d = ms[e.x];
  b_element_hess<T>(d, e.y);
}
// the Gram pass with the occupancy bounds of k_gram
template <typename T>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(gram_min_waves<T, false>(), gram_max_waves<T>())))
kb_gram(const DevMesh* __restrict__ ms, const int2* __restrict__ map) {
  const int2 e = map[blockIdx.x];
  const DevMesh d = ms[e.x];
  b_gram<T>(d, e.y);
}
EMU_BATCHED(kb_gram_reduce, kBlock, b_gram_reduce(d, e.y))
EMU_BATCHED(kb_control_a, kCtlThreads, b_control_a(d, e.y))
EMU_BATCHED(kb_uz, kBlock, b_uz(d, e.y))
EMU_BATCHED(kb_direction64, kBlock, b_direction<double>(d, e.y))
EMU_BATCHED(kb_direction32, kBlock, b_direction<float>(d, e.y))
EMU_BATCHED(kb_rhs, kBlock, b_rhs(d, e.y, 0, 1))
EMU_BATCHED(kb_fwd, kBlock, b_fwd(d, e.y, 1))
EMU_BATCHED(kb_bwd, kBlock, b_bwd(d, e.y, d.dq, 1))
EMU_BATCHED(kb_lscoef, kBlock, b_lscoef(d, e.y))
EMU_BATCHED(kb_control_b, kBlock, b_control_b(d, e.y))
EMU_BATCHED(kb_add_q, kBlock, b_add_q(d, e.y))
#undef EMU_BATCHED

// control blocks of every mesh of a batch into one contiguous array
__global__ void __launch_bounds__(64) kb_gather_ctl(const DevMesh* __restrict__ ms, int32_t* out) {
  constexpr int W = (int)(sizeof(Ctl) / 4);
  const int32_t* src = (const int32_t*)ms[blockIdx.x].ctl;
  for (int t = threadIdx.x; t < W; t += 64) out[(int64_t)W * blockIdx.x + t] = src[t];
}

static inline int blocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }
static inline int rhs_blocks(int64_t nf) { return blocks(nf * kRhsLanes); }
static inline int uz_blocks(int64_t n) { return blocks(n * kUzLanes); }

// Kernel instance for the mesh's precision and block structure.
typedef void (*MeshKernel)(DevMesh);
static MeshKernel pick_hess(const DevMesh& d) {
  return d.mixed ? (d.coupled ? k_element_hess<float, true> : k_element_hess<float, false>)
                 : (d.coupled ? k_element_hess<double, true> : k_element_hess<double, false>);
}
static MeshKernel pick_gram(const DevMesh& d) {
  return d.mixed ? (d.coupled ? k_gram<float, true> : k_gram<float, false>)
                 : (d.coupled ? k_gram<double, true> : k_gram<double, false>);
}
static MeshKernel pick_direction(const DevMesh& d) {
  return d.mixed ? (d.coupled ? k_direction<float, true> : k_direction<float, false>)
                 : (d.coupled ? k_direction<double, true> : k_direction<double, false>);
}
static MeshKernel pick_element(const DevMesh& d) { return d.mixed ? k_element<float> : k_element<double>; }
// The element pass and its Hessian blocks.  (One fused kernel was tried: at
// two waves per SIMD it spilled about 300 bytes per lane, and the pair ran
// 456 vs 331 us on the 1.5M-tet hinge limb.)
static void launch_element_pass(const DevMesh& d, hipStream_t st) {
  hipLaunchKernelGGL(pick_element(d), dim3(d.nb), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(pick_hess(d), dim3(d.nb), dim3(kBlock), 0, st, d);
}
static void launch_bone_blocks(const DevMesh& d, hipStream_t st) {
  if (d.nbones > 0)
    hipLaunchKernelGGL(d.mixed ? k_bone_blocks<float> : k_bone_blocks<double>, dim3(d.nbones), dim3(kBlock), 0, st, d);
}
static void launch_bone_dir(const DevMesh& d, hipStream_t st) {
  if (d.nbones > 0)
    hipLaunchKernelGGL(d.mixed ? k_bone_dir<float> : k_bone_dir<double>, dim3(d.nbones), dim3(kBlock), 0, st, d);
}
typedef void (*Pc1Kernel)(DevMesh, const double*, double*, double*, int);
typedef void (*Pc2Kernel)(DevMesh, const double*, double*, double*, const double*, int);
static Pc1Kernel pick_pc1(const DevMesh& d) {
  return d.mixed ? (d.coupled ? k_pc1<float, true> : k_pc1<float, false>)
                 : (d.coupled ? k_pc1<double, true> : k_pc1<double, false>);
}
static Pc2Kernel pick_pc2(const DevMesh& d) {
  return d.mixed ? (d.coupled ? k_pc2<float, true> : k_pc2<float, false>)
                 : (d.coupled ? k_pc2<double, true> : k_pc2<double, false>);
}

// Every bone tet takes its bone's representative (R, S): after a state is
// set from outside, each bone has one F.
__global__ void __launch_bounds__(kBlock) k_bone_sync(DevMesh d) {
  const int b = blockIdx.x, m = d.m;
  const int p0 = d.bone_ptr[b], p1 = d.bone_ptr[b + 1];
  const int rep = d.bone_el[p0];
  for (int q = p0 + 1 + threadIdx.x; q < p1; q += kBlock) {
    const int i = d.bone_el[q];
#pragma unroll
    for (int k = 0; k < 9; ++k) d.R[k * m + i] = d.R[k * m + rep];
#pragma unroll
    for (int k = 0; k < 6; ++k) d.S[k * m + i] = d.S[k * m + rep];
  }
}
void launch_bone_sync(const DevMesh& d, hipStream_t st) {
  if (d.nbones > 0) hipLaunchKernelGGL(k_bone_sync, dim3(d.nbones), dim3(kBlock), 0, st, d);
}

void launch_init_rest(const DevMesh& d, hipStream_t st) {
  hipLaunchKernelGGL(k_init_rest, dim3(blocks(d.m)), dim3(kBlock), 0, st, d);
}
void launch_set_F(const DevMesh& d, const double* F, const int32_t* eold, hipStream_t st) {
  hipLaunchKernelGGL(k_set_F, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, F, eold);
}
void launch_get_F(const DevMesh& d, double* F, const int32_t* eold, hipStream_t st) {
  hipLaunchKernelGGL(k_get_F, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, F, eold);
}
void launch_get_dir(const DevMesh& d, double* F, const int32_t* eold, hipStream_t st) {
  hipLaunchKernelGGL(k_get_dir, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, F, eold);
}
void launch_scatter_F(const DevMesh& d, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_F, dim3(blocks(d.m)), dim3(kBlock), 0, st, d);
}
void launch_solve(const DevMesh& d, const SolvePlan& pl, int add_pin, double* x, int check_done, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs, dim3(rhs_blocks(d.nf)), dim3(kBlock), 0, st, d, add_pin, check_done);
  for (int L = 0; L < pl.nlevels; ++L) launch_fwd_level(d, pl, L, check_done, st);
  for (int L = 0; L < pl.nlevels; ++L) launch_bwd_level(d, pl, L, x, check_done, st);
}
void launch_sweeps(const DevMesh& d, const SolvePlan& pl, double* x, hipStream_t st, int check_done) {
  for (int L = 0; L < pl.nlevels; ++L) launch_fwd_level(d, pl, L, check_done, st);
  for (int L = 0; L < pl.nlevels; ++L) launch_bwd_level(d, pl, L, x, check_done, st);
}
void launch_field_solve(const DevMesh& d, const SolvePlan& pl, const double* V, double* x, hipStream_t st,
                        int check_done) {
  hipLaunchKernelGGL(k_contrib_field, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, V, check_done);
  hipLaunchKernelGGL(k_rhs, dim3(rhs_blocks(d.nf)), dim3(kBlock), 0, st, d, 0, check_done);
  launch_sweeps(d, pl, x, st, check_done);
}
void launch_weighted_grad(const DevMesh& d, const double* x, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_weighted_grad, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, x, out);
}
void launch_hvp(const DevMesh& d, const double* V, const double* x, double* out, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_hvp, dim3(d.nb), dim3(kBlock), 0, st, d, V, x, out, part);
}
void launch_cg_update(const DevMesh& d, const double* P, const double* HP, double* lam, double* r, double* part,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_cg_update, dim3(d.nb), dim3(kBlock), 0, st, d, P, HP, lam, r, part);
}
void launch_cg_dir(const DevMesh& d, const double* Z, double* P, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_dir, dim3(d.nb), dim3(kBlock), 0, st, d, Z, P);
}
void launch_cg_scalar(const DevMesh& d, const double* part, int what, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kBlock), 0, st, d, part, what);
}
void launch_cg_begin(const DevMesh& d, int max_steps, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_begin, dim3(1), dim3(1), 0, st, d, max_steps);
}
void launch_precond(const DevMesh& d, const double* r, double* z, double* ypart, double* part, double* rbar,
                    hipStream_t st, int check_done) {
  hipLaunchKernelGGL(pick_pc1(d), dim3(d.nb), dim3(kBlock), 0, st, d, r, ypart, rbar, check_done);
  hipLaunchKernelGGL(k_pc_solve, dim3(1), dim3(kPcThreads), 0, st, d, ypart, check_done);
  hipLaunchKernelGGL(k_uz, dim3(uz_blocks(d.n)), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(pick_pc2(d), dim3(d.nb), dim3(kBlock), 0, st, d, r, z, part, (const double*)rbar, check_done);
}
void launch_cg_step(const DevMesh& d, const SolvePlan& pl, const CgWork& w, hipStream_t st) {
  launch_field_solve(d, pl, w.p, w.vx, st, 1);  // vx = L^{-1} G^T W p
  launch_hvp(d, w.p, w.vx, w.hp, w.part, st);
  launch_cg_scalar(d, w.part, kCgAlpha, st);
  launch_cg_update(d, w.p, w.hp, w.lam, w.r, w.part, st);
  launch_cg_scalar(d, w.part, kCgResid, st);
  launch_precond(d, w.r, w.z, w.ypart, w.part, w.rbar, st, 1);
  launch_cg_scalar(d, w.part, kCgBeta, st);
  launch_cg_dir(d, w.z, w.p, st);
}
void launch_grad_field(const DevMesh& d, const double* x, double* V, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_field, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, x, V);
}
void launch_lff_apply(const DevMesh& d, const double* x, double* V, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_field, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, x, V);
  hipLaunchKernelGGL(k_contrib_field, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, (const double*)V, 0);
  hipLaunchKernelGGL(k_rhs, dim3(rhs_blocks(d.nf)), dim3(kBlock), 0, st, d, 0, 0);
}
int eig_gram_blocks(int nf) { return std::max(1, std::min(512, (nf + 255) / 256)); }
void launch_eig_gram(int nf, int64_t pstride, const double* A, const double* B, double* part, double* out,
                     hipStream_t st) {
  const int nblk = eig_gram_blocks(nf);
  const int rows = (nf + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_eig_gram, dim3(nblk), dim3(kBlock), 0, st, nf, pstride, A, B, rows, part);
  hipLaunchKernelGGL(k_eig_reduce, dim3((kEigPairs + kBlock - 1) / kBlock), dim3(kBlock), 0, st, nblk, kEigPairs,
                     (const double*)part, out);
}
void launch_eig_mul(int nf, int64_t pstride, const double* Y, const double* W, double* X, hipStream_t st) {
  hipLaunchKernelGGL(k_eig_mul, dim3(blocks(nf)), dim3(kBlock), 0, st, nf, pstride, Y, W, X);
}
void launch_eig_resid(int nf, int64_t pstride, const double* X, const double* LX, const double* lam, int ncols,
                      double* part, double* out, hipStream_t st) {
  const int nblk = blocks(nf);
  hipLaunchKernelGGL(k_eig_resid, dim3(nblk), dim3(kBlock), 0, st, nf, pstride, X, LX, lam, ncols, part);
  hipLaunchKernelGGL(k_eig_reduce, dim3(1), dim3(kBlock), 0, st, nblk, ncols, (const double*)part, out);
}
int contact_blocks(const DevMesh& d) { return (d.nf + kBlock - 1) / kBlock; }
void launch_contact_force(const DevMesh& d, const double* obs, int np, int ns, double k, double* part,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_contact_force, dim3(std::max(1, contact_blocks(d))), dim3(kBlock), 0, st, d, obs, np, ns, k,
                     part);
}
void launch_contact_accum(const DevMesh& d, const double* x2, const double* z, double* zc, hipStream_t st) {
  const int64_t n = std::max(3 * (int64_t)d.nf, 9 * (int64_t)d.m);
  hipLaunchKernelGGL(k_contact_accum, dim3(blocks(n)), dim3(kBlock), 0, st, d, x2, z, zc);
}
void launch_accept_contact(const DevMesh& d, const double* zc, hipStream_t st) {
  hipLaunchKernelGGL(k_accept_contact, dim3(blocks(d.m)), dim3(kBlock), 0, st, d, zc);
  hipLaunchKernelGGL(k_clear_step, dim3(1), dim3(64), 0, st, d);
}
void launch_adj_da(const DevMesh& d, const double* lam, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_da, dim3(d.nb), dim3(kBlock), 0, st, d, lam, part);
}
void launch_group_sum(const DevMesh& d, const double* per, double scale, double* out, hipStream_t st) {
  if (d.ngroups > 0) hipLaunchKernelGGL(k_group_sum, dim3(d.ngroups), dim3(kBlock), 0, st, d, per, scale, out);
}

void launch_set_pins(const DevMesh& d, hipStream_t st) {
  hipLaunchKernelGGL(k_set_pins, dim3(blocks(d.npins)), dim3(kBlock), 0, st, d);
}

void launch_iteration(const DevMesh& d, const SolvePlan& pl, hipStream_t st) {
  launch_element_pass(d, st);
  launch_bone_blocks(d, st);
  hipLaunchKernelGGL(pick_gram(d), dim3(d.nbg), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_gram_reduce, dim3((kGramEntries + 15) / 16), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_control_a, dim3(1), dim3(kCtlThreads), 0, st, d);
  hipLaunchKernelGGL(k_uz, dim3(uz_blocks(d.n)), dim3(kBlock), 0, st, d);
  launch_bone_dir(d, st);
  hipLaunchKernelGGL(pick_direction(d), dim3(d.nb), dim3(kBlock), 0, st, d);
  launch_solve(d, pl, 0, d.dq, 1, st);
  hipLaunchKernelGGL(k_lscoef, dim3(d.nb), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_control_b, dim3(1), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_add_q, dim3(blocks(3 * (int64_t)d.nf)), dim3(kBlock), 0, st, d);
}

// One iteration with events between its phases: ev[0] element pass, ev[1]
// Woodbury correction, ev[2] ACAP solve of the direction, ev[3] line search,
// ev[4] end.
void launch_iteration_phased(const DevMesh& d, const SolvePlan& pl, hipStream_t st, hipEvent_t* ev) {
  (void)hipEventRecord(ev[0], st);
  launch_element_pass(d, st);
  (void)hipEventRecord(ev[1], st);
  launch_bone_blocks(d, st);
  hipLaunchKernelGGL(pick_gram(d), dim3(d.nbg), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_gram_reduce, dim3((kGramEntries + 15) / 16), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_control_a, dim3(1), dim3(kCtlThreads), 0, st, d);
  hipLaunchKernelGGL(k_uz, dim3(uz_blocks(d.n)), dim3(kBlock), 0, st, d);
  launch_bone_dir(d, st);
  hipLaunchKernelGGL(pick_direction(d), dim3(d.nb), dim3(kBlock), 0, st, d);
  (void)hipEventRecord(ev[2], st);
  launch_solve(d, pl, 0, d.dq, 1, st);
  (void)hipEventRecord(ev[3], st);
  hipLaunchKernelGGL(k_lscoef, dim3(d.nb), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_control_b, dim3(1), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_add_q, dim3(blocks(3 * (int64_t)d.nf)), dim3(kBlock), 0, st, d);
  (void)hipEventRecord(ev[4], st);
}

void launch_class(int k, const DevMesh& d, const SolvePlan& pl, hipStream_t st) {
  switch (k) {
    case 0:
      launch_element_pass(d, st);
      launch_bone_blocks(d, st);
      break;
    case 1: hipLaunchKernelGGL(pick_gram(d), dim3(d.nbg), dim3(kBlock), 0, st, d); break;
    case 2: hipLaunchKernelGGL(k_gram_reduce, dim3((kGramEntries + 15) / 16), dim3(kBlock), 0, st, d); break;
    case 3: hipLaunchKernelGGL(k_control_a, dim3(1), dim3(kCtlThreads), 0, st, d); break;
    case 4: hipLaunchKernelGGL(k_uz, dim3(uz_blocks(d.n)), dim3(kBlock), 0, st, d); break;
    case 5:
      launch_bone_dir(d, st);
      hipLaunchKernelGGL(pick_direction(d), dim3(d.nb), dim3(kBlock), 0, st, d);
      break;
    case 6: hipLaunchKernelGGL(k_rhs, dim3(rhs_blocks(d.nf)), dim3(kBlock), 0, st, d, 0, 1); break;
    case 7:
      for (int L = 0; L < pl.nlevels; ++L) launch_fwd_level(d, pl, L, 1, st);
      break;
    case 8:
      for (int L = 0; L < pl.nlevels; ++L) launch_bwd_level(d, pl, L, d.dq, 1, st);
      break;
    case 9: hipLaunchKernelGGL(k_lscoef, dim3(d.nb), dim3(kBlock), 0, st, d); break;
    case 10: hipLaunchKernelGGL(k_control_b, dim3(1), dim3(kBlock), 0, st, d); break;
    case 11: hipLaunchKernelGGL(k_add_q, dim3(blocks(3 * (int64_t)d.nf)), dim3(kBlock), 0, st, d); break;
    default: break;
  }
}

// evaluation at the current state: element pass, Woodbury system, direction
void launch_evaluate(const DevMesh& d, hipStream_t st) {
  launch_element_pass(d, st);
  launch_bone_blocks(d, st);
  hipLaunchKernelGGL(pick_gram(d), dim3(d.nbg), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_gram_reduce, dim3((kGramEntries + 15) / 16), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_control_a, dim3(1), dim3(kCtlThreads), 0, st, d);
  hipLaunchKernelGGL(k_uz, dim3(uz_blocks(d.n)), dim3(kBlock), 0, st, d);
  launch_bone_dir(d, st);
  hipLaunchKernelGGL(pick_direction(d), dim3(d.nb), dim3(kBlock), 0, st, d);
}

static inline void launch_map(void (*k)(const DevMesh*, const int2*), const BatchPlan& b, const BatchClass& c,
                              int threads, hipStream_t st) {
  if (c.count > 0) hipLaunchKernelGGL(k, dim3(c.count), dim3(threads), 0, st, b.meshes, b.map + c.offset);
}

void launch_batch_iteration(const BatchPlan& b, hipStream_t st) {
  if (b.n_meshes == 0) return;
  launch_map(b.mixed ? kb_element32 : kb_element64, b, b.element, kBlock, st);
  launch_map(b.mixed ? kb_element_hess<float> : kb_element_hess<double>, b, b.element, kBlock, st);
  launch_map(b.mixed ? kb_gram<float> : kb_gram<double>, b, b.gram, kBlock, st);
  launch_map(kb_gram_reduce, b, b.gram_reduce, kBlock, st);
  launch_map(kb_control_a, b, b.one, kCtlThreads, st);
  launch_map(kb_uz, b, b.uz, kBlock, st);
  launch_map(b.mixed ? kb_direction32 : kb_direction64, b, b.element, kBlock, st);
  launch_map(kb_rhs, b, b.rhs, kBlock, st);
  for (const auto& c : b.fwd) launch_map(kb_fwd, b, c, kBlock, st);
  for (const auto& c : b.bwd) launch_map(kb_bwd, b, c, kBlock, st);
  launch_map(kb_lscoef, b, b.element, kBlock, st);
  launch_map(kb_control_b, b, b.one, kBlock, st);
  launch_map(kb_add_q, b, b.add_q, kBlock, st);
}

void launch_batch_gather_ctl(const BatchPlan& b, int32_t* out, hipStream_t st) {
  if (b.n_meshes > 0) hipLaunchKernelGGL(kb_gather_ctl, dim3(b.n_meshes), dim3(64), 0, st, b.meshes, out);
}

void batch_layout(const std::vector<const DevMesh*>& ms, const std::vector<const SolvePlan*>& plans,
                  BatchPlan& b, std::vector<int2>& map) {
  map.clear();
  const int nm = (int)ms.size();
  b.n_meshes = nm;
  auto add = [&](BatchClass& c, auto count_of) {
    c.offset = (int64_t)map.size();
    for (int j = 0; j < nm; ++j) {
      const int cnt = count_of(j);
      for (int k = 0; k < cnt; ++k) map.push_back(make_int2(j, k));
    }
    c.count = (int)((int64_t)map.size() - c.offset);
  };
  add(b.element, [&](int j) { return ms[j]->nb; });
  add(b.gram, [&](int j) { return ms[j]->nbg; });
  add(b.gram_reduce, [&](int) { return (kGramEntries + 15) / 16; });
  add(b.one, [&](int) { return 1; });
  add(b.uz, [&](int j) { return uz_blocks(ms[j]->n); });
  add(b.rhs, [&](int j) { return rhs_blocks(ms[j]->nf); });
  add(b.add_q, [&](int j) { return blocks(3 * (int64_t)ms[j]->nf); });
  int nl = 0;
  for (int j = 0; j < nm; ++j) nl = std::max(nl, plans[j]->nlevels);
  b.fwd.assign(nl, BatchClass{});
  b.bwd.assign(nl, BatchClass{});
  for (int L = 0; L < nl; ++L) {
    BatchClass& c = b.fwd[L];
    c.offset = (int64_t)map.size();
    // column-form levels: one entry per group of four items
    for (int j = 0; j < nm; ++j)
      if (L < plans[j]->nlevels) {
        const int step = plans[j]->fwd_col[L] ? 4 : 1;
        for (int it = plans[j]->fwd_ptr[L]; it < plans[j]->fwd_ptr[L + 1]; it += step) map.push_back(make_int2(j, it));
      }
    c.count = (int)((int64_t)map.size() - c.offset);
  }
  for (int L = 0; L < nl; ++L) {
    BatchClass& c = b.bwd[L];
    c.offset = (int64_t)map.size();
    for (int j = 0; j < nm; ++j)
      if (L < plans[j]->nlevels)
        for (int it = plans[j]->bwd_ptr[L]; it < plans[j]->bwd_ptr[L + 1]; ++it) map.push_back(make_int2(j, it));
    c.count = (int)((int64_t)map.size() - c.offset);
  }
}

}  // namespace emu
