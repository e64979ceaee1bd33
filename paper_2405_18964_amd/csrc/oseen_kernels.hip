// Frequency-block matrices and the pieces of the Oseen block preconditioner.
//
// Both per-frequency systems of the method have the same 4x4 block pattern in
// the (v, lambda, p, mu) order of eq. (SubBlockG):
//   row 1:  a11 M v + (a12 M + b12 K + e12 N^T) lambda        + s B^T mu
//   row 2:  (a21 M + b21 K + e21 N) v + a22 M lambda          + s B^T p
//   row 3:  s B lambda
//   row 4:  s B v
// Stokes Z_j (section 3.2):  a11 = 1, a12 = a21 = c1, b12 = b21 = c2 nu,
//                            a22 = -1, e = 0, s = 1.
// Oseen G_j (eq. SubBlockG): a11 = tau, a12 = conj(d_j), b12 = tau nu,
//                            e12 = tau, a21 = d_j, b21 = tau nu, e21 = tau,
//                            a22 = -tau/beta, s = tau.
// Frequency vector layout as in inner_kernels.hip.
#include "kernels.h"

namespace pintoc {

// Velocity rows 1 and 2: Q2 tile kernel k_q2_block_vel (q2_tiles.hip).

// (B u)_k at Q1 node k for a velocity pair (ux, uy) on padded Q2 grids.
template <typename R>
__device__ inline void b_apply_node(const cpx<R>* __restrict__ ux, const cpx<R>* __restrict__ uy, int n, int k,
                                    double& sr, double& si) {
  const int nq = 2 * n + 1, np = n + 1;
  const double h = 1.0 / n;
  const int kx = k % np, ky = k / np;
  double mxx[5], gxx[5], mxy[5], gxy[5];
  mixed_rows(kx, n, h, mxx, gxx);
  mixed_rows(ky, n, h, mxy, gxy);
  sr = 0; si = 0;
  for (int dy = 0; dy < 5; ++dy) {
    const int jy = 2 * ky + dy - 2;
    if (jy < 0 || jy >= nq) continue;
    for (int dx = 0; dx < 5; ++dx) {
      const int jx = 2 * kx + dx - 2;
      if (jx < 0 || jx >= nq) continue;
      const double wa = mxy[dy] * gxx[dx], wb = gxy[dy] * mxx[dx];
      const cpx<R> a = ux[jy * nq + jx], c = uy[jy * nq + jx];
      sr -= wa * (double)a.x + wb * (double)c.x;
      si -= wa * (double)a.y + wb * (double)c.y;
    }
  }
}

// rows 3 and 4: yP[j][0] = s_j B lambda, yP[j][1] = s_j B v  (node 0 pinned: 0),
// s_j = bc[j].s
template <typename R>
__global__ __launch_bounds__(256) void k_block_pres(cpx<R>* __restrict__ yP, const cpx<R>* __restrict__ xV, int n,
                                                    const BlockCoef* __restrict__ bc, Mask mk) {
  const int nq2 = (2 * n + 1) * (2 * n + 1), np2 = (n + 1) * (n + 1);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int jb = blockIdx.y;
  if (k >= np2 || mk.off(jb)) return;
  const int b = jb & 1, j = jb >> 1;
  const size_t o = (size_t)jb * np2 + k;
  if (k == 0) { yP[o] = cmk<cpx<R>>(0, 0); return; }
  const cpx<R>* ux = xV + ((size_t)(j * 2 + (b == 0 ? 1 : 0)) * 2 + 0) * nq2;
  double sr, si;
  b_apply_node<R>(ux, ux + nq2, n, k, sr, si);
  const double s = bc[j].s;
  yP[o] = cmk<cpx<R>>(s * sr, s * si);
}

// Pressure inputs of the Schur step of Algorithm 3:
//   out[j][0] = in[j][0] - tau_j B y2_j,   out[j][1] = in[j][1] - tau_j B y1_j
// with y1, y2 given as 2-component velocity batches [j][comp] (node 0 -> 0).
template <typename R>
__global__ __launch_bounds__(256) void k_schur_rhs(cpx<R>* __restrict__ out, const cpx<R>* __restrict__ in,
                                                   const cpx<R>* __restrict__ y1, const cpx<R>* __restrict__ y2,
                                                   int n, const double* __restrict__ ftau, Mask mk) {
  const int nq2 = (2 * n + 1) * (2 * n + 1), np2 = (n + 1) * (n + 1);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int jb = blockIdx.y;
  if (k >= np2 || mk.off(jb)) return;
  const int b = jb & 1, j = jb >> 1;
  const size_t o = (size_t)jb * np2 + k;
  if (k == 0) { out[o] = cmk<cpx<R>>(0, 0); return; }
  const cpx<R>* u = (b == 0 ? y2 : y1) + (size_t)j * 2 * nq2;
  double sr, si;
  b_apply_node<R>(u, u + nq2, n, k, sr, si);
  const double tau = ftau[j];
  const cpx<R> v = in[o];
  out[o] = cmk<cpx<R>>((double)v.x - tau * sr, (double)v.y - tau * si);
}

// u-step of the Oseen Schur inverse on the unconstrained Q1 grid:
//   with z1 = zz[j][1], z2 = zz[j][0] (already multiplied by (tau M_N)^{-1}),
//   U[j][0] = u2 = (d M + tau L) z1 - tau/beta M z2
//   U[j][1] = u1 = tau M z1 + (conj(d) M + tau L^T) z2,   L = nu K + N,
// with the frequency's own tau, beta, nu (ftau, fbeta, fnu).
template <typename R>
__global__ __launch_bounds__(256) void k_oseen_hp(cpx<R>* __restrict__ U, const cpx<R>* __restrict__ zz, int n,
                                                  const double2* __restrict__ dj, const double* __restrict__ ftau,
                                                  const double* __restrict__ fbeta, const double* __restrict__ fnu,
                                                  const double* __restrict__ conv, Mask mk) {
  const int np = n + 1, np2 = np * np;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (k >= np2 || mk.off(j)) return;
  const int ix = k % np, iy = k / np;
  const double h = 1.0 / n;
  double mx[3], kx[3], my[3], ky[3];
  q1_rows(ix, n, h, mx, kx);
  q1_rows(iy, n, h, my, ky);
  const cpx<R>* z2 = zz + (size_t)(j * 2 + 0) * np2;
  const cpx<R>* z1 = zz + (size_t)(j * 2 + 1) * np2;
  const double* cn = conv ? conv + (size_t)k * 18 : nullptr;
  double M1[2] = {0, 0}, K1[2] = {0, 0}, N1[2] = {0, 0}, M2[2] = {0, 0}, K2[2] = {0, 0}, T2[2] = {0, 0};
  for (int dy = 0; dy < 3; ++dy) {
    const int jy = iy + dy - 1;
    if (jy < 0 || jy > n) continue;
    for (int dx = 0; dx < 3; ++dx) {
      const int jx = ix + dx - 1;
      if (jx < 0 || jx > n) continue;
      const double wm = mx[dx] * my[dy], wk = kx[dx] * my[dy] + mx[dx] * ky[dy];
      const cpx<R> a = z1[jy * np + jx], c = z2[jy * np + jx];
      M1[0] += wm * (double)a.x; M1[1] += wm * (double)a.y;
      K1[0] += wk * (double)a.x; K1[1] += wk * (double)a.y;
      M2[0] += wm * (double)c.x; M2[1] += wm * (double)c.y;
      K2[0] += wk * (double)c.x; K2[1] += wk * (double)c.y;
      if (cn) {
        const double wn = cn[dy * 3 + dx], wt = cn[9 + dy * 3 + dx];
        N1[0] += wn * (double)a.x; N1[1] += wn * (double)a.y;
        T2[0] += wt * (double)c.x; T2[1] += wt * (double)c.y;
      }
    }
  }
  const double2 d = dj[j];
  const double tau = ftau[j], beta = fbeta[j], nu = fnu[j];
  const double u2r = d.x * M1[0] - d.y * M1[1] + tau * (nu * K1[0] + N1[0]) - (tau / beta) * M2[0];
  const double u2i = d.x * M1[1] + d.y * M1[0] + tau * (nu * K1[1] + N1[1]) - (tau / beta) * M2[1];
  const double u1r = tau * M1[0] + d.x * M2[0] + d.y * M2[1] + tau * (nu * K2[0] + T2[0]);
  const double u1i = tau * M1[1] + d.x * M2[1] - d.y * M2[0] + tau * (nu * K2[1] + T2[1]);
  U[(size_t)(j * 2 + 0) * np2 + k] = cmk<cpx<R>>(u2r, u2i);
  U[(size_t)(j * 2 + 1) * np2 + k] = cmk<cpx<R>>(u1r, u1i);
}

// Copy between the frequency-vector velocity layout V[j][b][comp] and a
// contiguous per-block batch X[j][comp] (dir 0: V -> X, dir 1: X -> V).
template <typename R>
__global__ __launch_bounds__(256) void k_block_copy(cpx<R>* __restrict__ V, cpx<R>* __restrict__ X, int nq2, int b,
                                                    int dir, Mask mk) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  const int jc = blockIdx.y;                    // j * 2 + comp
  if (node >= nq2 || mk.off(jc)) return;
  const int comp = jc & 1, j = jc >> 1;
  const size_t ov = ((size_t)(j * 2 + b) * 2 + comp) * nq2 + node;
  const size_t ox = (size_t)jc * nq2 + node;
  if (dir == 0) X[ox] = V[ov];
  else V[ov] = X[ox];
}

// out = c0 A + c1 f_j B + c2 C (real coefficients; B or C may be null; f_j =
// c1f[frequency of the grid], 1 when c1f is null); out may alias A.
template <typename R>
__global__ __launch_bounds__(256) void k_combine3(cpx<R>* out, const cpx<R>* A, const cpx<R>* B, const cpx<R>* C,
                                                  double c0, double c1, double c2, const double* __restrict__ c1f,
                                                  size_t n, int seg, Mask mk) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int grid = (int)(e / seg);
    if (mk.off(grid)) continue;
    const cpx<R> a = A[e];
    double r = c0 * (double)a.x, i = c0 * (double)a.y;
    if (B) {
      const double cb = c1f ? c1 * c1f[grid / mk.fpj] : c1;
      const cpx<R> v = B[e];
      r += cb * (double)v.x;
      i += cb * (double)v.y;
    }
    if (C) { const cpx<R> v = C[e]; r += c2 * (double)v.x; i += c2 * (double)v.y; }
    out[e] = cmk<cpx<R>>(r, i);
  }
}

template <typename R>
void launch_block_mat(hipStream_t s, cpx<R>* yV, cpx<R>* yP, const cpx<R>* xV, const cpx<R>* xP, int n, int nf,
                      const BlockCoef* bc, const R* tcN, const R* tcNT, Mask mk) {
  const int np2 = (n + 1) * (n + 1);
  launch_q2_block_vel<R>(s, yV, xV, xP, n, nf, bc, tcN, tcNT, mk);
  hipLaunchKernelGGL(k_block_pres<R>, dim3((np2 + 255) / 256, 2 * nf), dim3(256), 0, s, yP, xV, n, bc, mk);
}

template <typename R>
void launch_schur_rhs(hipStream_t s, cpx<R>* out, const cpx<R>* in, const cpx<R>* y1, const cpx<R>* y2, int n,
                      int nf, const double* ftau, Mask mk) {
  const int np2 = (n + 1) * (n + 1);
  hipLaunchKernelGGL(k_schur_rhs<R>, dim3((np2 + 255) / 256, 2 * nf), dim3(256), 0, s, out, in, y1, y2, n, ftau, mk);
}

template <typename R>
void launch_oseen_hp(hipStream_t s, cpx<R>* U, const cpx<R>* zz, int n, int nf, const double2* dj, const double* ftau,
                     const double* fbeta, const double* fnu, const double* conv, Mask mk) {
  const int np2 = (n + 1) * (n + 1);
  hipLaunchKernelGGL(k_oseen_hp<R>, dim3((np2 + 255) / 256, nf), dim3(256), 0, s, U, zz, n, dj, ftau, fbeta, fnu,
                     conv, mk);
}

template <typename R>
void launch_block_copy(hipStream_t s, cpx<R>* V, cpx<R>* X, int n, int nf, int b, int dir, Mask mk) {
  const int nq2 = (2 * n + 1) * (2 * n + 1);
  hipLaunchKernelGGL(k_block_copy<R>, dim3((nq2 + 255) / 256, 2 * nf), dim3(256), 0, s, V, X, nq2, b, dir, mk);
}

template <typename R>
void launch_combine3(hipStream_t s, cpx<R>* out, const cpx<R>* A, const cpx<R>* B, const cpx<R>* C, double c0,
                     double c1, double c2, const double* c1f, size_t n, int seg, Mask mk) {
  hipLaunchKernelGGL(k_combine3<R>, dim3(2048), dim3(256), 0, s, out, A, B, C, c0, c1, c2, c1f, n, seg, mk);
}

#define PINTOC_OSEEN_INST(R)                                                                                       \
  template void launch_block_mat<R>(hipStream_t, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*, int, int,         \
                                    const BlockCoef*, const R*, const R*, Mask);                               \
  template void launch_schur_rhs<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, int, int,   \
                                    const double*, Mask);                                                                \
  template void launch_oseen_hp<R>(hipStream_t, cpx<R>*, const cpx<R>*, int, int, const double2*, const double*,   \
                                   const double*, const double*, const double*, Mask);                                   \
  template void launch_block_copy<R>(hipStream_t, cpx<R>*, cpx<R>*, int, int, int, int, Mask);                           \
  template void launch_combine3<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, double,      \
                                   double, double, const double*, size_t, int, Mask);

PINTOC_OSEEN_INST(double)
PINTOC_OSEEN_INST(float)

}  // namespace pintoc
