// Shared device/host helpers of the pintoc library (gfx950).
//
// Discretisation (section 2.2): Q2 velocity / Q1 pressure Taylor-Hood
// elements on N x N uniform squares of [0,1]^2.  On a uniform tensor grid
// every operator of the method is a short sum of Kronecker products of 1-D
// matrices, so the kernels evaluate rows of
//   M2 = M1 (x) M1,  K2 = K1 (x) M1 + M1 (x) K1          (Q2, Q1 alike)
//   Bx = -(mix (x) gmix),  By = -(gmix (x) mix)           (Q1 rows, Q2 cols)
// from the 1-D element matrices below (x fastest, so the right factor acts
// along x).  Velocity grids are stored padded: (2N+1)^2 nodes with the
// Dirichlet boundary held at zero; pressure grids hold all (N+1)^2 nodes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pintoc {

// ----------------------------------------------------------------- complex
template <typename R> struct cpx_t;
template <> struct cpx_t<double> { using type = double2; };
template <> struct cpx_t<float> { using type = float2; };
template <typename R> using cpx = typename cpx_t<R>::type;

template <typename C> __host__ __device__ inline C cmk(double re, double im) {
  C c; c.x = re; c.y = im; return c;
}
__host__ __device__ inline double2 operator+(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 operator-(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 operator*(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__host__ __device__ inline float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 operator*(float s, float2 a) { return make_float2(s * a.x, s * a.y); }

template <typename C> __host__ __device__ inline C cmul(C a, C b) {
  C c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c;
}
template <typename C> __host__ __device__ inline C cconj(C a) { C c; c.x = a.x; c.y = -a.y; return c; }
// a / b
template <typename C> __host__ __device__ inline C cdiv(C a, C b) {
  auto den = b.x * b.x + b.y * b.y;
  C c; c.x = (a.x * b.x + a.y * b.y) / den; c.y = (a.y * b.x - a.x * b.y) / den; return c;
}
// i * a
template <typename C> __host__ __device__ inline C cmuli(C a) { C c; c.x = -a.y; c.y = a.x; return c; }

// ---------------------------------------------------- 1-D element matrices
// Quadratic Lagrange element on [0, h], nodes 0, h/2, h:
//   mass = h/30 [[4,2,-1],[2,16,2],[-1,2,4]],  stiffness = 1/(3h) [[7,-8,1],[-8,16,-8],[1,-8,7]].
// Linear element on [0, h]: mass = h/6 [[2,1],[1,2]], stiffness = 1/h [[1,-1],[-1,1]].
// Mixed (rows P1 psi_a, columns P2 phi_b):
//   int psi_a phi_b   = h [[1/6, 1/3, 0], [0, 1/3, 1/6]]
//   int psi_a phi_b'  =   [[-5/6, 2/3, 1/6], [-1/6, -2/3, 5/6]]

// Row of the assembled 1-D Q2 mass/stiffness at node i, for column offsets
// -2..2 (index o+2).  Valid for interior nodes 1 <= i <= 2n-1 (all the kernels
// need); a vertex node (i even) sees two elements, a midpoint node one.
__host__ __device__ inline void q2_rows(int i, double h, double m[5], double k[5]) {
  const double sm = h / 30.0, sk = 1.0 / (3.0 * h);
  if ((i & 1) == 0) {
    m[0] = -1 * sm; m[1] = 2 * sm; m[2] = 8 * sm; m[3] = 2 * sm; m[4] = -1 * sm;
    k[0] = 1 * sk; k[1] = -8 * sk; k[2] = 14 * sk; k[3] = -8 * sk; k[4] = 1 * sk;
  } else {
    m[0] = 0; m[1] = 2 * sm; m[2] = 16 * sm; m[3] = 2 * sm; m[4] = 0;
    k[0] = 0; k[1] = -8 * sk; k[2] = 16 * sk; k[3] = -8 * sk; k[4] = 0;
  }
}

// Row of the assembled 1-D Q1 mass/stiffness at node i in [0, n] (natural
// boundary conditions), column offsets -1..1 (index o+1).
__host__ __device__ inline void q1_rows(int i, int n, double h, double m[3], double k[3]) {
  const double sm = h / 6.0, sk = 1.0 / h;
  const bool lo = i > 0, hi = i < n;           // element to the left / right exists
  m[0] = lo ? 1 * sm : 0.0;
  m[2] = hi ? 1 * sm : 0.0;
  m[1] = (lo ? 2 * sm : 0.0) + (hi ? 2 * sm : 0.0);
  k[0] = lo ? -1 * sk : 0.0;
  k[2] = hi ? -1 * sk : 0.0;
  k[1] = (lo ? sk : 0.0) + (hi ? sk : 0.0);
}

// Mixed rows for pressure node k in [0, n]: Q2 column offsets -2..2 around
// Q2 node 2k.  mix = int psi_k phi_j, gmix = int psi_k phi_j'.
__host__ __device__ inline void mixed_rows(int k, int n, double h, double mx[5], double gx[5]) {
  const bool lo = k > 0, hi = k < n;
  // element k-1 (psi_1 row) covers offsets -2..0, element k (psi_0 row) covers 0..2
  mx[0] = 0.0;
  mx[1] = lo ? h / 3.0 : 0.0;
  mx[2] = (lo ? h / 6.0 : 0.0) + (hi ? h / 6.0 : 0.0);
  mx[3] = hi ? h / 3.0 : 0.0;
  mx[4] = 0.0;
  gx[0] = lo ? -1.0 / 6.0 : 0.0;
  gx[1] = lo ? -2.0 / 3.0 : 0.0;
  gx[2] = (lo ? 5.0 / 6.0 : 0.0) + (hi ? -5.0 / 6.0 : 0.0);
  gx[3] = hi ? 2.0 / 3.0 : 0.0;
  gx[4] = hi ? 1.0 / 6.0 : 0.0;
}

// Column view of the mixed matrices: for Q2 node j (any, 0..2n) the Q1 rows k
// that touch it are k = floor(j/2) - 1 + q, q = 0..2 (out-of-range k give 0).
// Returns mix[k][j] and gmix[k][j] for those three k.
__host__ __device__ inline void mixed_cols(int j, int n, double h, double mx[3], double gx[3]) {
  const int k0 = (j >> 1) - 1;
  for (int q = 0; q < 3; ++q) {
    const int k = k0 + q;
    mx[q] = 0.0; gx[q] = 0.0;
    if (k < 0 || k > n) continue;
    const int off = j - 2 * k;                 // -2..2 when coupled
    if (off < -2 || off > 2) continue;
    double a[5], b[5];
    mixed_rows(k, n, h, a, b);
    mx[q] = a[off + 2]; gx[q] = b[off + 2];
  }
}

// ------------------------------------------------------------ coefficients
// A scalar operator  alpha M + gamma K + eta N + etat N^T  on one grid family.
// Complex coefficients; for the Stokes operators only the real parts are
// nonzero.  N (convection) is applied from per-node stencil tables.
struct OpCoef {
  double2 alpha, gamma, eta, etat;
};

// Coefficients of one frequency block in the (v, lambda, p, mu) pattern shared
// by the Stokes Z_j and the Oseen G_j (see oseen_kernels.hip).
struct BlockCoef {
  double2 a11, a12, b12, e12, a21, b21, e21, a22;
  double s, pad;
};

// Per-frequency activity mask of a batched launch: grid f of the batch belongs
// to frequency f / fpj; a frequency whose entry is 0 is skipped (its blocks
// return at once).  m == nullptr: every grid is active.
struct Mask {
  const int* m;
  int fpj;
  __device__ bool off(int f) const { return m != nullptr && m[f / fpj] == 0; }
};

inline __host__ __device__ int q2n(int n) { return 2 * n + 1; }
inline __host__ __device__ int q1n(int n) { return n + 1; }

}  // namespace pintoc
