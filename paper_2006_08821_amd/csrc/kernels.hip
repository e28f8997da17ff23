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

#include "device.hpp"
#include "kernels.hpp"

namespace emu {

#define DEV __device__ __forceinline__

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

// Block-wide reduction of NV double-double values (kBlock threads); result valid
// in thread 0.  Fixed tree order.
template <int NV>
DEV void block_reduce_dd(DD (&v)[NV], DD* sh) {
  const int t = threadIdx.x;
  for (int k = 0; k < NV; ++k) sh[k * kBlock + t] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s)
      for (int k = 0; k < NV; ++k) sh[k * kBlock + t] = dd_add(sh[k * kBlock + t], sh[k * kBlock + t + s]);
    __syncthreads();
  }
  if (t == 0)
    for (int k = 0; k < NV; ++k) v[k] = sh[k * kBlock];
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
          T theta = (A[qq][qq] - A[pp][pp]) / (T(2) * apq);
          T t = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
          T c = T(1) / sqrt(t * t + T(1)), s = t * c;
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
template <typename T, int N>
DEV bool chol_packed(const T (&A)[N][N], T* L) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T s = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j * (j + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
    if (!(s > T(0))) return false;
    T d = sqrt(s);
    L[j * (j + 1) / 2 + j] = d;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
      L[i * (i + 1) / 2 + j] = t / d;
    }
  }
  return true;
}
template <typename T, int N>
DEV void chol_solve(const T* L, T* x) {  // in place: L L^T x = b
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T t = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[i * (i + 1) / 2 + k] * x[k];
    x[i] = t / L[i * (i + 1) / 2 + i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    T t = x[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) t -= L[k * (k + 1) / 2 + i] * x[k];
    x[i] = t / L[i * (i + 1) / 2 + i];
  }
}
template <typename T, int N>
DEV void chol_lt_mul(const T* L, const T* x, T* y) {  // y = L^T x
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T t = 0;
#pragma unroll
    for (int k = i; k < N; ++k) t += L[k * (k + 1) / 2 + i] * x[k];
    y[i] = t;
  }
}

// Make A positive semi-definite (eigenvalues < 0 -> 0) unless a Cholesky
// factorization already succeeds; then add beta I and factor.  Returns 1 if
// the clamp changed A.
template <typename T, int N>
DEV int clamp_add_factor(T (&A)[N][N], T beta, T* L) {
  int clamped = 0;
  if (!chol_packed<T, N>(A, L)) {
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
    clamped = 1;
  }
#pragma unroll
  for (int k = 0; k < N; ++k) A[k][k] += beta;
  if (!chol_packed<T, N>(A, L)) {
    // beta > 0 makes this positive definite; guard against beta == 0 with a tiny shift
    T sc = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) sc = A[k][k] > sc ? A[k][k] : sc;
#pragma unroll
    for (int k = 0; k < N; ++k) A[k][k] += T(1e-12) * sc + T(1e-300);
    chol_packed<T, N>(A, L);
  }
  return clamped;
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
__global__ void __launch_bounds__(kBlock) k_rhs(DevMesh d, int add_pin, int check_done) {
  if (check_done && d.ctl->done) return;
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= d.nf) return;
  double acc[3] = {0, 0, 0};
  if (add_pin)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = d.pin_rhs[3 * f + c];
  for (int k = d.inc_ptr[f]; k < d.inc_ptr[f + 1]; ++k) {
    int code = d.inc[k];
    const double* src = d.contrib + (int64_t)12 * (code >> 2) + 3 * (code & 3);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += src[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) d.rhs[3 * f + c] = acc[c];
}

// Forward sweep of one level.  Work item (s, r0): rows [r0, r0 + kTriRows) of
// supernode s.  Frontal vector f = [rhs at the columns; 0] + children's update
// vectors; rows r < w give y = Linv f_top, rows r >= w give u = f_r - M_r f_top.
__global__ void __launch_bounds__(kBlock) k_fwd(DevMesh d, int it0, int check_done) {
  if (check_done && d.ctl->done) return;
  __shared__ double ft[kMaxFrontW * 3];
  const int2 item = d.fwd_items[it0 + blockIdx.x];
  const int s = item.x, r0 = item.y;
  const int w = d.sn_w[s], h = d.sn_h[s], col0 = d.sn_col0[s];
  const int fo = d.sn_front[s];
  const int t = threadIdx.x;
  for (int c = t; c < w; c += kBlock) {
    double a0 = d.rhs[3 * (col0 + c)], a1 = d.rhs[3 * (col0 + c) + 1], a2 = d.rhs[3 * (col0 + c) + 2];
    for (int k = d.gptr[fo + c]; k < d.gptr[fo + c + 1]; ++k) {
      const double* u = d.upd + 3 * (int64_t)d.gsrc[k];
      a0 += u[0];
      a1 += u[1];
      a2 += u[2];
    }
    ft[3 * c] = a0;
    ft[3 * c + 1] = a1;
    ft[3 * c + 2] = a2;
  }
  __syncthreads();
  const int lane = t & 63, wave = t >> 6;
  const double* V = d.vals + d.sn_valoff[s];
  const int64_t tri = (int64_t)w * (w + 1) / 2;
  for (int rr = wave; rr < kTriRows; rr += kBlock / 64) {
    const int r = r0 + rr;
    if (r >= h) break;
    const double* row = r < w ? V + (int64_t)r * (r + 1) / 2 : V + tri + (int64_t)(r - w) * w;
    const int len = r < w ? r + 1 : w;
    double a0 = 0, a1 = 0, a2 = 0;
    for (int c = lane; c < len; c += 64) {
      double v = row[c];
      a0 += v * ft[3 * c];
      a1 += v * ft[3 * c + 1];
      a2 += v * ft[3 * c + 2];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
      a2 += __shfl_xor(a2, off);
    }
    if (lane == 0) {
      if (r < w) {
        d.ybuf[3 * (col0 + r)] = a0;
        d.ybuf[3 * (col0 + r) + 1] = a1;
        d.ybuf[3 * (col0 + r) + 2] = a2;
      } else {
        double b0 = 0, b1 = 0, b2 = 0;
        for (int k = d.gptr[fo + r]; k < d.gptr[fo + r + 1]; ++k) {
          const double* u = d.upd + 3 * (int64_t)d.gsrc[k];
          b0 += u[0];
          b1 += u[1];
          b2 += u[2];
        }
        double* o = d.upd + 3 * (int64_t)(d.sn_rowoff[s] + r - w);
        o[0] = b0 - a0;
        o[1] = b1 - a1;
        o[2] = b2 - a2;
      }
    }
  }
}

// Backward sweep of one level.  Work item (s, c0): columns [c0, c0 + kTriRows)
// of supernode s:  x_c = sum_{r >= c, r < w} Linv[r][c] y_r - sum_r' M[r'][c] x[rows_r'].
__global__ void __launch_bounds__(kBlock) k_bwd(DevMesh d, int it0, double* x, int check_done) {
  if (check_done && d.ctl->done) return;
  constexpr int CH = 1024;
  __shared__ double z[CH * 3];
  __shared__ double part[kBlock / 64][64][3];
  const int2 item = d.bwd_items[it0 + blockIdx.x];
  const int s = item.x, c0 = item.y;
  const int w = d.sn_w[s], h = d.sn_h[s], col0 = d.sn_col0[s];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int c = c0 + lane;
  const double* V = d.vals + d.sn_valoff[s];
  const int64_t tri = (int64_t)w * (w + 1) / 2;
  const int32_t* rows = d.rows + d.sn_rowoff[s];
  double a0 = 0, a1 = 0, a2 = 0;
  for (int base = c0; base < h; base += CH) {
    const int nr = min(CH, h - base);
    __syncthreads();
    for (int k = t; k < nr; k += kBlock) {
      const int r = base + k;
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
    if (c < w) {
      for (int k = wave; k < nr; k += kBlock / 64) {
        const int r = base + k;
        double v;
        if (r < w)
          v = (c <= r) ? V[(int64_t)r * (r + 1) / 2 + c] : 0.0;
        else
          v = V[tri + (int64_t)(r - w) * w + c];
        a0 += v * z[3 * k];
        a1 += v * z[3 * k + 1];
        a2 += v * z[3 * k + 2];
      }
    }
  }
  part[wave][lane][0] = a0;
  part[wave][lane][1] = a1;
  part[wave][lane][2] = a2;
  __syncthreads();
  if (wave == 0 && c < w) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double sum = part[0][lane][k];
#pragma unroll
      for (int ww = 1; ww < kBlock / 64; ++ww) sum += part[ww][lane][k];
      x[3 * (col0 + c) + k] = sum;
    }
  }
}

// q = solution at free vertices, pin targets at pinned vertices
__global__ void __launch_bounds__(kBlock) k_set_pins(DevMesh d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.npins) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) d.q[3 * (d.nf + i) + c] = d.pin_xyz[3 * i + c];
}

__global__ void __launch_bounds__(kBlock) k_add_q(DevMesh d) {
  if (d.ctl->done) return;
  const double sg = d.ctl->sigma;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * d.nf) return;
  d.q[i] += sg * d.dq[i];
}

// --------------------------------------------------------------- element pass
// Accept the previous step (if sigma > 0): X = S + sigma D(p), R <- R polar(X),
// S <- sym(polar(X)^T X).  Then at the new state: energy, exact gradient
// G = vol P(F) + beta (F - A) (eq. gradient), the two clamped Hessian blocks
// + beta I, their Cholesky factors and gbar = H^{-1} g.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_element(DevMesh d) {
  Ctl* ctl = d.ctl;
  if (ctl->done) return;
  __shared__ DD sh[2 * kBlock];
  __shared__ int shc[2][kBlock];
  const double sigma = ctl->sigma;
  DD acc[2] = {DD{0, 0}, DD{0, 0}};
  int nclamp = 0, ninv = 0;
  const int m = d.m;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    Elem e;
    load_elem(d, i, e);
    double R[9], S[9];
    load_R(d, i, R);
    load_S(d, i, S);
    if (sigma != 0.0) {
      double py[9], D[9], X[9], Rx[9], Rn[9], Sn[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) py[k] = d.p[k * m + i];
      from_y<double>(py, D);
#pragma unroll
      for (int k = 0; k < 9; ++k) X[k] = S[k] + sigma * D[k];
      polar3(X, Rx);
      matmul3(R, Rx, Rn);
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
    acc[0] = dd_add_d(acc[0], e.vol * psi + 0.5 * beta * dres);
    ninv += (J <= 0.0);
    const double kap = e.lhat * (J - 1.0) - e.mu;
    double G[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        G[3 * a + b] = e.vol * (e.mu * S[3 * a + b] + kap * C[3 * a + b] + 2.0 * afk * Su[a] * e.u[b]) +
                       beta * (S[3 * a + b] - At[3 * a + b]);
    double gn = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) gn += G[k] * G[k];
    acc[1] = dd_add_d(acc[1], gn);
    double gy[9];
    to_y<double, double>(G, gy);
    // Hessian blocks in the rotated basis (precision T)
    T St[9], ut[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) St[k] = (T)S[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) ut[k] = (T)e.u[k];
    const T muT = (T)e.mu, kapT = (T)kap, phiT = (T)(2.0 * afk), volT = (T)e.vol, lhT = (T)e.lhat;
    T cy[9];
    to_y<T, double>(C, cy);
    T Hs[6][6], Hk[3][3];
#pragma unroll
    for (int y = 0; y < 6; ++y)
#pragma unroll
      for (int z = 0; z < 6; ++z)
        Hs[y][z] = volT * (hproj<T>(y, z, St, muT, kapT, phiT, ut) + lhT * cy[y] * cy[z]);
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int z = 0; z < 3; ++z) Hk[y][z] = volT * hproj<T>(6 + y, 6 + z, St, muT, kapT, phiT, ut);
    T Ls[21], Lk[6];
    nclamp += clamp_add_factor<T, 6>(Hs, (T)beta, Ls);
    nclamp += clamp_add_factor<T, 3>(Hk, (T)beta, Lk);
    T gs[6], gk[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) gs[k] = (T)gy[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) gk[k] = (T)gy[6 + k];
    chol_solve<T, 6>(Ls, gs);
    chol_solve<T, 3>(Lk, gk);
    T* gbar = (T*)d.gbar;
    T* Lf = (T*)d.Lf;
#pragma unroll
    for (int k = 0; k < 6; ++k) gbar[k * m + i] = gs[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) gbar[(6 + k) * m + i] = gk[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) Lf[k * m + i] = Ls[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) Lf[(21 + k) * m + i] = Lk[k];
  }
  block_reduce_dd<2>(acc, sh);
  shc[0][threadIdx.x] = nclamp;
  shc[1][threadIdx.x] = ninv;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      shc[0][threadIdx.x] += shc[0][threadIdx.x + s];
      shc[1][threadIdx.x] += shc[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    d.part_e[2 * blockIdx.x] = acc[0].hi;
    d.part_e[2 * blockIdx.x + 1] = acc[0].lo;
    d.part_g[2 * blockIdx.x] = acc[1].hi;
    d.part_g[2 * blockIdx.x + 1] = acc[1].lo;
    d.part_cnt[2 * blockIdx.x] = shc[0][0];
    d.part_cnt[2 * blockIdx.x + 1] = shc[1][0];
  }
}

// --------------------------------------------------------------- Woodbury Gram
// Per element: Z = T H^{-1} T^T (9x9, F coordinates; T = (R (x) I) Y) and the
// mode gradients gphi_j = sum_v phi_j(v) b_v.  Accumulates, per workgroup,
//   Gram[(c,j),(c',j')] += w^2 gphi_j^T Z_{cc'} gphi_j'   (6 pairs c <= c')
//   y[(c,j)]            += w (R D(gbar) gphi_j)[c]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gram(DevMesh d) {
  if (d.ctl->done) return;
  constexpr int TE = 64;
  __shared__ T zs[TE][45];
  __shared__ T gp[TE][kMaxK1][3];
  __shared__ T fg[TE][9];
  __shared__ T ws[TE];
  const int t = threadIdx.x;
  const int m = d.m;
  const int per = (m + d.nbg - 1) / d.nbg;
  const int e0 = blockIdx.x * per, e1 = min(m, e0 + per);
  const int jj = t >> 4, jp = t & 15;
  const int k1 = d.k1;
  T acc[6] = {0, 0, 0, 0, 0, 0};
  T accy = 0;
  const int yc = t >> 4, yj = t & 15;  // for t < 48
  for (int base = e0; base < e1; base += TE) {
    const int ne = min(TE, e1 - base);
    __syncthreads();
    if (t < ne) {
      const int i = base + t;
      double R[9];
      load_R(d, i, R);
      const T* Lf = (const T*)d.Lf;
      const T* gbar = (const T*)d.gbar;
      T Ls[21], Lk[6];
#pragma unroll
      for (int k = 0; k < 21; ++k) Ls[k] = Lf[k * m + i];
#pragma unroll
      for (int k = 0; k < 6; ++k) Lk[k] = Lf[(21 + k) * m + i];
      // columns of T: vec(R Y_y), y = 0..8
      T Tm[9][9];
#pragma unroll
      for (int y = 0; y < 9; ++y) {
        double Yy[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        Yy[kYi[y][0]] += kYv[y][0];
        if (kYn[y] > 1) Yy[kYi[y][1]] += kYv[y][1];
        double RY[9];
        matmul3(R, Yy, RY);
#pragma unroll
        for (int k = 0; k < 9; ++k) Tm[k][y] = (T)RY[k];
      }
      // N = T L^{-T} per block: rows n solve n L^T = t  (forward substitution)
      T N[9][9];
#pragma unroll
      for (int r = 0; r < 9; ++r) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          T v = Tm[r][j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= N[r][k] * Ls[j * (j + 1) / 2 + k];
          N[r][j] = v / Ls[j * (j + 1) / 2 + j];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          T v = Tm[r][6 + j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= N[r][6 + k] * Lk[j * (j + 1) / 2 + k];
          N[r][6 + j] = v / Lk[j * (j + 1) / 2 + j];
        }
      }
      int o = 0;
#pragma unroll
      for (int a = 0; a < 9; ++a)
#pragma unroll
        for (int b = a; b < 9; ++b) {
          T s = 0;
#pragma unroll
          for (int k = 0; k < 9; ++k) s += N[a][k] * N[b][k];
          zs[t][o++] = s;
        }
      T gb[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) gb[k] = gbar[k * m + i];
      double gbd[9], D[9], RD[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) gbd[k] = (double)gb[k];
      from_y<double>(gbd, D);
      matmul3(R, D, RD);
#pragma unroll
      for (int k = 0; k < 9; ++k) fg[t][k] = (T)RD[k];
      ws[t] = (T)d.w[i];
    }
    // mode gradients, all threads
    for (int idx = t; idx < ne * kMaxK1; idx += kBlock) {
      const int el = idx / kMaxK1, j = idx % kMaxK1;
      const int i = base + el;
      T g0 = 0, g1 = 0, g2 = 0;
      if (j < k1) {
        double b[4][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) b[k][c] = d.dminv[(3 * k + c) * m + i];
#pragma unroll
        for (int c = 0; c < 3; ++c) b[3][c] = -(b[0][c] + b[1][c] + b[2][c]);
        double a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          double ph = d.phi[(int64_t)kMaxK1 * d.vid[k * m + i] + j];
          a0 += ph * b[k][0];
          a1 += ph * b[k][1];
          a2 += ph * b[k][2];
        }
        g0 = (T)a0;
        g1 = (T)a1;
        g2 = (T)a2;
      }
      gp[el][j][0] = g0;
      gp[el][j][1] = g1;
      gp[el][j][2] = g2;
    }
    __syncthreads();
    // accumulate
    for (int el = 0; el < ne; ++el) {
      const T w2 = ws[el] * ws[el];
      const T gj[3] = {gp[el][jj][0], gp[el][jj][1], gp[el][jj][2]};
      const T gq[3] = {gp[el][jp][0], gp[el][jp][1], gp[el][jp][2]};
      int pair = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int cp = c; cp < 3; ++cp) {
          T s = 0;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            T hz = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const int A = 3 * c + a, B = 3 * cp + b;
              const int lo = A < B ? A : B, hi = A < B ? B : A;
              const int zi = lo * 9 - lo * (lo - 1) / 2 + (hi - lo);
              hz += zs[el][zi] * gq[b];
            }
            s += gj[a] * hz;
          }
          acc[pair++] += w2 * s;
        }
      if (t < 48) {
        accy += ws[el] * (fg[el][3 * yc] * gp[el][yj][0] + fg[el][3 * yc + 1] * gp[el][yj][1] +
                          fg[el][3 * yc + 2] * gp[el][yj][2]);
      }
    }
  }
  double* out = d.part_gram + (int64_t)kGramEntries * blockIdx.x;
#pragma unroll
  for (int pr = 0; pr < 6; ++pr) out[pr * 256 + t] = (double)acc[pr];
  if (t < 48) out[1536 + t] = (double)accy;
}

__global__ void __launch_bounds__(kBlock) k_gram_reduce(DevMesh d) {
  if (d.ctl->done) return;
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= kGramEntries) return;
  double s = 0;
  for (int b = 0; b < d.nbg; ++b) s += d.part_gram[(int64_t)b * kGramEntries + e];
  d.gram[e] = s;
}

// Single workgroup: reduce energy / gradient-norm partials, test convergence,
// then build C = Lambda - alpha Gram (3k1 x 3k1), Cholesky, z = C^{-1} y.
__global__ void __launch_bounds__(kBlock) k_control_a(DevMesh d) {
  Ctl* ctl = d.ctl;
  if (ctl->done) return;
  __shared__ DD sh[2 * kBlock];
  __shared__ double Cm[48][49];
  __shared__ double yv[48];
  __shared__ int flag;
  const int t = threadIdx.x;
  DD acc[2] = {DD{0, 0}, DD{0, 0}};
  int cl = 0, inv = 0;
  for (int b = t; b < d.nb; b += kBlock) {
    acc[0] = dd_add(acc[0], DD{d.part_e[2 * b], d.part_e[2 * b + 1]});
    acc[1] = dd_add(acc[1], DD{d.part_g[2 * b], d.part_g[2 * b + 1]});
  }
  block_reduce_dd<2>(acc, sh);
  if (t == 0) {
    for (int b = 0; b < d.nb; ++b) {
      cl += d.part_cnt[2 * b];
      inv += d.part_cnt[2 * b + 1];
    }
    const double g2 = acc[1].hi + acc[1].lo;
    ctl->energy = acc[0].hi + acc[0].lo;
    ctl->gnorm2 = g2;
    ctl->clamped = cl;
    ctl->inverted = inv;
    if (ctl->iter == 0 && ctl->gnorm0_2 < 0) ctl->gnorm0_2 = g2;
    int stop = 0;
    if (!(g2 == g2) || !(ctl->energy == ctl->energy) || g2 > 1e300) {
      ctl->status = EMU_E_NONFINITE_CODE;
      stop = 1;
    } else if (!ctl->eval_only && g2 <= ctl->tol2) {
      ctl->status = 0;
      stop = 1;
    } else if (!ctl->eval_only && ctl->iter >= ctl->max_iters) {
      ctl->status = EMU_E_NOT_CONVERGED_CODE;
      stop = 1;
    }
    flag = stop;
  }
  __syncthreads();
  if (flag) {
    if (t == 0) ctl->done = 1;
    return;
  }
  const int k1 = d.k1, K = 3 * k1;
  if (K == 0) {
    return;
  }
  // C[(c,j),(c',j')] in compact indices (c*k1 + j)
  for (int idx = t; idx < K * K; idx += kBlock) {
    const int r = idx / K, q = idx % K;
    const int c = r / k1, j = r % k1, cp = q / k1, jp = q % k1;
    double g;
    if (c <= cp) {
      const int pair = c == 0 ? cp : (c == 1 ? 2 + cp : 5);
      g = d.gram[pair * 256 + j * 16 + jp];
    } else {
      const int pair = cp == 0 ? c : (cp == 1 ? 2 + c : 5);
      g = d.gram[pair * 256 + jp * 16 + j];
    }
    Cm[r][q] = (r == q ? d.nu[j] : 0.0) - d.alpha * g;
  }
  for (int r = t; r < K; r += kBlock) yv[r] = d.gram[1536 + (r / k1) * 16 + (r % k1)];
  __syncthreads();
  // symmetrize, then right-looking Cholesky in place (lower)
  for (int idx = t; idx < K * K; idx += kBlock) {
    const int r = idx / K, q = idx % K;
    if (r > q) {
      double v = 0.5 * (Cm[r][q] + Cm[q][r]);
      Cm[r][q] = v;
    }
  }
  if (t == 0) flag = 0;
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    if (t == 0) {
      double v = Cm[j][j];
      if (!(v > 0)) flag = 1;
      Cm[j][j] = v > 0 ? sqrt(v) : 1.0;
    }
    __syncthreads();
    for (int i = j + 1 + t; i < K; i += kBlock) Cm[i][j] /= Cm[j][j];
    __syncthreads();
    for (int idx = t; idx < (K - j - 1) * (K - j - 1); idx += kBlock) {
      const int i = j + 1 + idx / (K - j - 1), k = j + 1 + idx % (K - j - 1);
      if (k <= i) Cm[i][k] -= Cm[i][j] * Cm[k][j];
    }
    __syncthreads();
  }
  if (t == 0) {
    double zz[48];
    if (flag) {
      for (int r = 0; r < K; ++r) zz[r] = 0.0;
      ctl->chol_fail += 1;
    } else {
      for (int i = 0; i < K; ++i) {
        double s = yv[i];
        for (int k = 0; k < i; ++k) s -= Cm[i][k] * zz[k];
        zz[i] = s / Cm[i][i];
      }
      for (int i = K - 1; i >= 0; --i) {
        double s = zz[i];
        for (int k = i + 1; k < K; ++k) s -= Cm[k][i] * zz[k];
        zz[i] = s / Cm[i][i];
      }
    }
    for (int c = 0; c < 3; ++c)
      for (int j = 0; j < kMaxK1; ++j) d.zbuf[c * kMaxK1 + j] = j < k1 ? zz[c * k1 + j] : 0.0;
  }
}

// uz[v][c] = sum_j z[(c,j)] phi_j(v)  (zero at pinned vertices)
__global__ void __launch_bounds__(kBlock) k_uz(DevMesh d) {
  if (d.ctl->done) return;
  int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= d.n) return;
  double a[3] = {0, 0, 0};
  if (d.k1 > 0) {
    const double* ph = d.phi + (int64_t)kMaxK1 * v;
#pragma unroll
    for (int j = 0; j < kMaxK1; ++j) {
      double p = ph[j];
#pragma unroll
      for (int c = 0; c < 3; ++c) a[c] += d.zbuf[c * kMaxK1 + j] * p;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) d.uz[3 * v + c] = a[c];
}

// Direction: d = gbar + alpha H^{-1} B^T z with B^T z = w Y^T vec(R^T G uz);
// p = -d; g.p = (L^T gbar).(L^T p) per block; contributions of dF = R D(p).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_direction(DevMesh d) {
  Ctl* ctl = d.ctl;
  if (ctl->done) return;
  __shared__ DD sh[kBlock];
  DD acc[1] = {DD{0, 0}};
  const int m = d.m;
  const T* Lf = (const T*)d.Lf;
  const T* gbar = (const T*)d.gbar;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
    Elem e;
    load_elem(d, i, e);
    double R[9], Az[9], RA[9];
    load_R(d, i, R);
    gather_grad(d.uz, e, Az);
    matTmul3(R, Az, RA);
    T ty[9];
    to_y<T, double>(RA, ty);
    T Ls[21], Lk[6], gb[9];
#pragma unroll
    for (int k = 0; k < 21; ++k) Ls[k] = Lf[k * m + i];
#pragma unroll
    for (int k = 0; k < 6; ++k) Lk[k] = Lf[(21 + k) * m + i];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      gb[k] = gbar[k * m + i];
      ty[k] *= (T)e.w;
    }
    chol_solve<T, 6>(Ls, ty);
    chol_solve<T, 3>(Lk, ty + 6);
    double p[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      p[k] = -((double)gb[k] + d.alpha * (double)ty[k]);
      d.p[k * m + i] = p[k];
    }
    // g . p
    T pt[9], a1[9], a2[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) pt[k] = (T)p[k];
    chol_lt_mul<T, 6>(Ls, gb, a1);
    chol_lt_mul<T, 3>(Lk, gb + 6, a1 + 6);
    chol_lt_mul<T, 6>(Ls, pt, a2);
    chol_lt_mul<T, 3>(Lk, pt + 6, a2 + 6);
    double gp = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) gp += (double)a1[k] * (double)a2[k];
    acc[0] = dd_add_d(acc[0], gp);
    double D[9], dF[9];
    from_y<double>(p, D);
    matmul3(R, D, dF);
    write_contrib(d, i, e, dF);
  }
  block_reduce_dd<1>(acc, sh);
  if (threadIdx.x == 0) {
    d.part_ls[2 * kLsTerms * blockIdx.x + 12] = acc[0].hi;
    d.part_ls[2 * kLsTerms * blockIdx.x + 13] = acc[0].lo;
  }
}

// Line-search polynomial: E(sigma) - E(0) = sum_k c_k sigma^k (k = 1..6), exact
// per element along F(sigma) = R (S + sigma D), A(sigma) = A + sigma dA.
__global__ void __launch_bounds__(kBlock) k_lscoef(DevMesh d) {
  Ctl* ctl = d.ctl;
  if (ctl->done) return;
  __shared__ DD sh[6 * kBlock];
  DD acc[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) acc[k] = DD{0, 0};
  const int m = d.m;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += d.nb * kBlock) {
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
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = dd_add_d(acc[k], c[k]);
  }
  block_reduce_dd<6>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      d.part_ls[2 * kLsTerms * blockIdx.x + 2 * k] = acc[k].hi;
      d.part_ls[2 * kLsTerms * blockIdx.x + 2 * k + 1] = acc[k].lo;
    }
}

// Single workgroup: Armijo backtracking on the exact polynomial (Algorithm 1).
__global__ void __launch_bounds__(kBlock) k_control_b(DevMesh d) {
  Ctl* ctl = d.ctl;
  if (ctl->done) return;
  __shared__ DD sh[kLsTerms * kBlock];
  const int t = threadIdx.x;
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
  const double gtp = acc[6].hi + acc[6].lo;
  ctl->gtp = gtp;
  ctl->solves += 1;
  if (!(gtp < 0.0)) {
    // no descent (|g| at the rounding floor): stop, keeping the state
    ctl->status = ctl->stall_rel > 0 ? 0 : EMU_E_LINESEARCH_CODE;
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
    const double g2 = ctl->gnorm2, g02 = ctl->gnorm0_2;
    const bool stalled = ctl->stall_rel > 0 && g2 <= ctl->stall_rel * ctl->stall_rel * g02;
    ctl->status = stalled ? 0 : EMU_E_LINESEARCH_CODE;
    ctl->done = 1;
  }
}

// ------------------------------------------------------------------ launch helpers
static inline int blocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

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
  hipLaunchKernelGGL(k_rhs, dim3(blocks(d.nf)), dim3(kBlock), 0, st, d, add_pin, check_done);
  for (int L = 0; L < pl.nlevels; ++L) {
    int n0 = pl.fwd_ptr[L], n1 = pl.fwd_ptr[L + 1];
    if (n1 > n0) hipLaunchKernelGGL(k_fwd, dim3(n1 - n0), dim3(kBlock), 0, st, d, n0, check_done);
  }
  for (int L = 0; L < pl.nlevels; ++L) {
    int n0 = pl.bwd_ptr[L], n1 = pl.bwd_ptr[L + 1];
    if (n1 > n0) hipLaunchKernelGGL(k_bwd, dim3(n1 - n0), dim3(kBlock), 0, st, d, n0, x, check_done);
  }
}
void launch_set_pins(const DevMesh& d, hipStream_t st) {
  hipLaunchKernelGGL(k_set_pins, dim3(blocks(d.npins)), dim3(kBlock), 0, st, d);
}

void launch_iteration(const DevMesh& d, const SolvePlan& pl, hipStream_t st) {
  if (d.mixed) {
    hipLaunchKernelGGL(k_element<float>, dim3(d.nb), dim3(kBlock), 0, st, d);
    hipLaunchKernelGGL(k_gram<float>, dim3(d.nbg), dim3(kBlock), 0, st, d);
  } else {
    hipLaunchKernelGGL(k_element<double>, dim3(d.nb), dim3(kBlock), 0, st, d);
    hipLaunchKernelGGL(k_gram<double>, dim3(d.nbg), dim3(kBlock), 0, st, d);
  }
  hipLaunchKernelGGL(k_gram_reduce, dim3(blocks(kGramEntries)), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_control_a, dim3(1), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_uz, dim3(blocks(d.n)), dim3(kBlock), 0, st, d);
  if (d.mixed)
    hipLaunchKernelGGL(k_direction<float>, dim3(d.nb), dim3(kBlock), 0, st, d);
  else
    hipLaunchKernelGGL(k_direction<double>, dim3(d.nb), dim3(kBlock), 0, st, d);
  launch_solve(d, pl, 0, d.dq, 1, st);
  hipLaunchKernelGGL(k_lscoef, dim3(d.nb), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_control_b, dim3(1), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_add_q, dim3(blocks(3 * (int64_t)d.nf)), dim3(kBlock), 0, st, d);
}

void launch_class(int k, const DevMesh& d, const SolvePlan& pl, hipStream_t st) {
  switch (k) {
    case 0:
      if (d.mixed) hipLaunchKernelGGL(k_element<float>, dim3(d.nb), dim3(kBlock), 0, st, d);
      else hipLaunchKernelGGL(k_element<double>, dim3(d.nb), dim3(kBlock), 0, st, d);
      break;
    case 1:
      if (d.mixed) hipLaunchKernelGGL(k_gram<float>, dim3(d.nbg), dim3(kBlock), 0, st, d);
      else hipLaunchKernelGGL(k_gram<double>, dim3(d.nbg), dim3(kBlock), 0, st, d);
      break;
    case 2: hipLaunchKernelGGL(k_gram_reduce, dim3(blocks(kGramEntries)), dim3(kBlock), 0, st, d); break;
    case 3: hipLaunchKernelGGL(k_control_a, dim3(1), dim3(kBlock), 0, st, d); break;
    case 4: hipLaunchKernelGGL(k_uz, dim3(blocks(d.n)), dim3(kBlock), 0, st, d); break;
    case 5:
      if (d.mixed) hipLaunchKernelGGL(k_direction<float>, dim3(d.nb), dim3(kBlock), 0, st, d);
      else hipLaunchKernelGGL(k_direction<double>, dim3(d.nb), dim3(kBlock), 0, st, d);
      break;
    case 6: hipLaunchKernelGGL(k_rhs, dim3(blocks(d.nf)), dim3(kBlock), 0, st, d, 0, 1); break;
    case 7:
      for (int L = 0; L < pl.nlevels; ++L) {
        int n0 = pl.fwd_ptr[L], n1 = pl.fwd_ptr[L + 1];
        if (n1 > n0) hipLaunchKernelGGL(k_fwd, dim3(n1 - n0), dim3(kBlock), 0, st, d, n0, 1);
      }
      break;
    case 8:
      for (int L = 0; L < pl.nlevels; ++L) {
        int n0 = pl.bwd_ptr[L], n1 = pl.bwd_ptr[L + 1];
        if (n1 > n0) hipLaunchKernelGGL(k_bwd, dim3(n1 - n0), dim3(kBlock), 0, st, d, n0, d.dq, 1);
      }
      break;
    case 9: hipLaunchKernelGGL(k_lscoef, dim3(d.nb), dim3(kBlock), 0, st, d); break;
    case 10: hipLaunchKernelGGL(k_control_b, dim3(1), dim3(kBlock), 0, st, d); break;
    case 11: hipLaunchKernelGGL(k_add_q, dim3(blocks(3 * (int64_t)d.nf)), dim3(kBlock), 0, st, d); break;
    default: break;
  }
}

// evaluation at the current state: element pass, Woodbury system, direction
void launch_evaluate(const DevMesh& d, hipStream_t st) {
  if (d.mixed) {
    hipLaunchKernelGGL(k_element<float>, dim3(d.nb), dim3(kBlock), 0, st, d);
    hipLaunchKernelGGL(k_gram<float>, dim3(d.nbg), dim3(kBlock), 0, st, d);
  } else {
    hipLaunchKernelGGL(k_element<double>, dim3(d.nb), dim3(kBlock), 0, st, d);
    hipLaunchKernelGGL(k_gram<double>, dim3(d.nbg), dim3(kBlock), 0, st, d);
  }
  hipLaunchKernelGGL(k_gram_reduce, dim3(blocks(kGramEntries)), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_control_a, dim3(1), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_uz, dim3(blocks(d.n)), dim3(kBlock), 0, st, d);
  if (d.mixed)
    hipLaunchKernelGGL(k_direction<float>, dim3(d.nb), dim3(kBlock), 0, st, d);
  else
    hipLaunchKernelGGL(k_direction<double>, dim3(d.nb), dim3(kBlock), 0, st, d);
}

}  // namespace emu
