// Outer Krylov method in the frequency domain (section 3.1, Theorem 1): the
// all-at-once matrix is the block-circulant preconditioner plus a corner
// term, A = P_C + U, so in the Fourier basis A^ = diag(G_j) + F U F^{-1} acts
// on the kept frequencies without any FFT: per-frequency blocks G_j plus two
// time samples (v at the last step, lambda at the first) spread over all
// frequencies.
//
// Outer frequency vector (FP64): V[j][b][comp][(2N+1)^2] then P[j][b][(N+1)^2]
// (complex), each frequency scaled by s_j = sqrt(w_j / nt) with w_0 = w_{nt/2}
// = 1 and w_j = 2 otherwise.  With this scaling the Euclidean inner product of
// the stored reals equals the time-domain one (Parseval with the conjugate
// half folded in), so the Krylov method is the time-domain one in another
// orthonormal basis.
#include "kernels.h"

namespace pintoc {

// y[j] = f[j] x[j] over the V and P parts (in place allowed)
__global__ __launch_bounds__(256) void k_freq_scale(double2* __restrict__ y, const double2* __restrict__ x,
                                                    const double* __restrict__ f, int nf, int segV, int segP) {
  const size_t n = (size_t)nf * (segV + segP);
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t vV = (size_t)nf * segV;
    const int j = e < vV ? (int)(e / segV) : (int)((e - vV) / segP);
    const double a = f[j];
    const double2 v = x[e];
    y[e] = make_double2(a * v.x, a * v.y);
  }
}

// FP64 outer vector -> inner-precision block vectors (dir 0), applying
// T_l^{-1} for Stokes (mode 1); or inner block solution -> FP64 outer vector
// (dir 1), applying T_r^{-1} (mode 1).  tj[j] = (d_c, c2).  One thread per
// (frequency, component, node) of the velocity and (frequency, node) of the
// pressure, handling the pair b = 0, 1.
template <typename R>
__global__ __launch_bounds__(256) void k_freq_convert(const double2* __restrict__ xo, cpx<R>* __restrict__ V,
                                                      cpx<R>* __restrict__ P, double2* __restrict__ yo, int nf,
                                                      int nq2, int np2, const double2* __restrict__ tj, double tau,
                                                      int mode, int dir) {
  const size_t nv = (size_t)nf * 2 * nq2, np = (size_t)nf * np2;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nv + np) return;
  const bool vel = e < nv;
  int j;
  size_t i0, i1;                          // positions of b = 0 and b = 1 (same in every layout)
  if (vel) {
    j = (int)(e / (2 * (size_t)nq2));
    const size_t r = e - (size_t)j * 2 * nq2;          // comp * nq2 + node
    const int comp = (int)(r / nq2), node = (int)(r - (size_t)comp * nq2);
    i0 = ((size_t)(j * 2 + 0) * 2 + comp) * nq2 + node;
    i1 = ((size_t)(j * 2 + 1) * 2 + comp) * nq2 + node;
  } else {
    const size_t q = e - nv;
    j = (int)(q / np2);
    const int node = (int)(q - (size_t)j * np2);
    i0 = (size_t)nf * 4 * nq2 + (size_t)(j * 2 + 0) * np2 + node;
    i1 = (size_t)nf * 4 * nq2 + (size_t)(j * 2 + 1) * np2 + node;
  }
  const double st = sqrt(tau);
  const double dc = tj[j].x, c2 = tj[j].y;
  const size_t off = (size_t)nf * 4 * nq2;            // start of the P part of the outer vector
  if (dir == 0) {
    double2 X0 = xo[i0], X1 = xo[i1];
    if (mode == 1) {
      const double2 idr = make_double2(dc * X0.y / tau, -dc * X0.x / tau);   // -i dc X0 / tau
      if (vel) {
        const double2 s2 = (c2 / st) * (X1 + idr);
        X0 = (1.0 / st) * X0;
        X1 = s2;
      } else {
        const double2 s4 = (1.0 / st) * (X1 + idr);
        X0 = (1.0 / (st * c2)) * X0;
        X1 = s4;
      }
    }
    if (vel) { V[i0] = cmk<cpx<R>>(X0.x, X0.y); V[i1] = cmk<cpx<R>>(X1.x, X1.y); }
    else { P[i0 - off] = cmk<cpx<R>>(X0.x, X0.y); P[i1 - off] = cmk<cpx<R>>(X1.x, X1.y); }
  } else {
    cpx<R> a, b;
    if (vel) { a = V[i0]; b = V[i1]; }
    else { a = P[i0 - off]; b = P[i1 - off]; }
    double2 Y0 = make_double2((double)a.x, (double)a.y), Y1 = make_double2((double)b.x, (double)b.y);
    if (mode == 1) {
      if (vel) {
        const double2 y2 = (c2 / st) * Y1;
        const double2 y1 = (1.0 / st) * (Y0 + make_double2(-dc * y2.y / st, dc * y2.x / st));
        Y0 = y1; Y1 = y2;
      } else {
        const double2 y4 = (1.0 / st) * Y1;
        const double2 y3 = (1.0 / (st * c2)) * (Y0 + make_double2(-dc * c2 * y4.y / st, dc * c2 * y4.x / st));
        Y0 = y3; Y1 = y4;
      }
    }
    yo[i0] = Y0;
    yo[i1] = Y1;
  }
}

// Time samples of the velocity fields from a scaled outer vector:
//   v_{nt-1} = sum_j s_j Re(v~_j e^{2 pi i j (nt-1)/nt}),  lambda_0 = sum_j s_j Re(lambda~_j),
// out[0..1] = v_{nt-1} (comp x, y), out[2..3] = lambda_0, each (2N+1)^2 reals.
__global__ __launch_bounds__(256) void k_freq_corner_gather(const double2* __restrict__ xV, double* __restrict__ out,
                                                            const double* __restrict__ sj, int nf, int nt, int nq2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * nq2) return;
  const int comp = e / nq2, node = e - comp * nq2;
  double v = 0.0, l = 0.0;
  for (int j = 0; j < nf; ++j) {
    const double2 a = xV[((size_t)(j * 2 + 0) * 2 + comp) * nq2 + node];
    const double2 b = xV[((size_t)(j * 2 + 1) * 2 + comp) * nq2 + node];
    double sn, cs;
    sincospi(2.0 * (double)j * (double)(nt - 1) / (double)nt, &sn, &cs);
    v += sj[j] * (a.x * cs - a.y * sn);
    l += sj[j] * b.x;
  }
  out[(size_t)comp * nq2 + node] = v;
  out[(size_t)(2 + comp) * nq2 + node] = l;
}

// M applied to the four real fields of k_freq_corner_gather (Q2 mass on
// interior nodes, zero on the boundary): out[f] = M in[f].
__global__ __launch_bounds__(256) void k_freq_corner_mass(const double* __restrict__ in, double* __restrict__ out,
                                                          int n) {
  const int nq = 2 * n + 1, nq2 = nq * nq;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 4 * nq2) return;
  const int f = e / nq2, node = e - f * nq2;
  const int ix = node % nq, iy = node / nq;
  double v = 0.0;
  if (ix > 0 && iy > 0 && ix < nq - 1 && iy < nq - 1) {
    double mx[5], kx[5], my[5], ky[5];
    const double h = 1.0 / n;
    q2_rows(ix, h, mx, kx);
    q2_rows(iy, h, my, ky);
    const double* u = in + (size_t)f * nq2;
    for (int dy = 0; dy < 5; ++dy) {
      const int jy = iy + dy - 2;
      if (jy < 0 || jy >= nq) continue;
      double s = 0.0;
      for (int dx = 0; dx < 5; ++dx) {
        const int jx = ix + dx - 2;
        if (jx < 0 || jx >= nq) continue;
        s += mx[dx] * u[jy * nq + jx];
      }
      v += my[dy] * s;
    }
  }
  out[(size_t)f * nq2 + node] = v;
}

// y~_j += s_j M v_{nt-1} on the state rows (b = 1) and
// y~_j += s_j e^{2 pi i j / nt} M lambda_0 on the adjoint rows (b = 0).
__global__ __launch_bounds__(256) void k_freq_corner_apply(double2* __restrict__ yV, const double* __restrict__ mf,
                                                           const double* __restrict__ sj, int nf, int nt, int nq2) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)nf * 2 * nq2) return;
  const int j = (int)(e / (2 * (size_t)nq2));
  const int r = (int)(e - (size_t)j * 2 * nq2);
  const int comp = r / nq2, node = r - comp * nq2;
  const double mv = mf[(size_t)comp * nq2 + node], ml = mf[(size_t)(2 + comp) * nq2 + node];
  double sn, cs;
  sincospi(2.0 * (double)j / (double)nt, &sn, &cs);
  const double s = sj[j];
  double2& ys = yV[((size_t)(j * 2 + 1) * 2 + comp) * nq2 + node];
  ys.x += s * mv;
  double2& ya = yV[((size_t)(j * 2 + 0) * 2 + comp) * nq2 + node];
  ya.x += s * cs * ml;
  ya.y += s * sn * ml;
}

void launch_freq_scale(hipStream_t s, double2* y, const double2* x, const double* f, int nf, int segV, int segP) {
  hipLaunchKernelGGL(k_freq_scale, dim3(2048), dim3(256), 0, s, y, x, f, nf, segV, segP);
}

template <typename R>
void launch_freq_convert(hipStream_t s, const double2* xo, cpx<R>* V, cpx<R>* P, double2* yo, int nf, int nq2,
                         int np2, const double2* tj, double tau, int mode, int dir) {
  const size_t n = (size_t)nf * (2 * nq2 + np2);
  hipLaunchKernelGGL(k_freq_convert<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xo, V, P, yo, nf, nq2, np2,
                     tj, tau, mode, dir);
}

void launch_freq_corner(hipStream_t s, double2* yV, const double2* xV, double* tmp, const double* sj, int n, int nf,
                        int nt) {
  const int nq2 = (2 * n + 1) * (2 * n + 1);
  hipLaunchKernelGGL(k_freq_corner_gather, dim3((2 * nq2 + 255) / 256), dim3(256), 0, s, xV, tmp, sj, nf, nt, nq2);
  hipLaunchKernelGGL(k_freq_corner_mass, dim3((4 * nq2 + 255) / 256), dim3(256), 0, s, tmp, tmp + (size_t)4 * nq2, n);
  const size_t m = (size_t)nf * 2 * nq2;
  hipLaunchKernelGGL(k_freq_corner_apply, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, yV,
                     tmp + (size_t)4 * nq2, sj, nf, nt, nq2);
}

template void launch_freq_convert<double>(hipStream_t, const double2*, double2*, double2*, double2*, int, int, int,
                                          const double2*, double, int, int);
template void launch_freq_convert<float>(hipStream_t, const double2*, float2*, float2*, double2*, int, int, int,
                                         const double2*, double, int, int);

}  // namespace pintoc
