// Block Fourier transform in time (section 3.1) fused with the frequency-
// block transforms of the Stokes factorisation G_j = T_l Z_j T_r (section 3.2).
//
// Forward: for every level index n (a velocity or pressure node of one time
// level), the two real sequences r[b=0][t][n] and r[b=1][t][n], t = 0..nt-1,
// are packed as z_t = r0 + i r1 and transformed with one complex radix-2 FFT
// (forward kernel exp(-2 pi i j t / nt), unnormalised).  Their spectra are
// separated by Hermitian symmetry:
//   R0_j = (Z_j + conj(Z_{nt-j})) / 2,   R1_j = (Z_j - conj(Z_{nt-j})) / (2i)
// and only j = 0..nt/2 are kept (real data, so R_{nt-j} = conj(R_j)).
// A work-group loads a tile [t = 0..nt-1] x [TN consecutive n] (coalesced along
// n), transforms in LDS and writes [j][TN consecutive n] (coalesced along n).
//
// Frequency-domain layout:  V[j][b][comp][(2N+1)^2], P[j][b][(N+1)^2] (complex).
#include "kernels.h"

namespace pintoc {

__device__ inline int bitrev(int v, int logn) { return (int)(__brev((unsigned)v) >> (32 - logn)); }

// Radix-2 decimation-in-time stages over TN sequences of length nt held in
// LDS in bit-reversed order.  sgn = -1 forward, +1 inverse (twiddle conj).
__device__ inline void lds_fft(double2* buf, int TN, int nt, int logn, const double2* __restrict__ tw, bool inverse) {
  const int half = nt >> 1;
  for (int s = 0; s < logn; ++s) {
    const int m = 1 << s;
    for (int e = threadIdx.x; e < TN * half; e += blockDim.x) {
      const int n = e / half, k = e - n * half;
      const int pos = k & (m - 1);
      const int i0 = ((k >> s) << (s + 1)) + pos, i1 = i0 + m;
      double2 w = tw[pos << (logn - 1 - s)];
      if (inverse) w.y = -w.y;
      double2* q = buf + n * nt;
      const double2 a = q[i0], b = cmul(q[i1], w);
      q[i0] = a + b;
      q[i1] = a - b;
    }
    __syncthreads();
  }
}

// mode 0: plain transform (Oseen blocks);  mode 1: apply T_l^{-1} (Stokes).
// tj[j] = (d_c, c2) per kept frequency.
template <typename R>
__global__ __launch_bounds__(256) void k_time_fft_fwd(const double* __restrict__ r, cpx<R>* __restrict__ V, cpx<R>* __restrict__ P,
                               int nt, int logn, int L, int nq2, int np2, int nf, int TN,
                               const double2* __restrict__ tw, const double2* __restrict__ tj, double tau, int mode) {
  extern __shared__ double2 buf[];
  const int n0 = blockIdx.x * TN;
  for (int e = threadIdx.x; e < TN * nt; e += blockDim.x) {
    const int n = e % TN, t = e / TN;
    double a = 0, b = 0;
    if (n0 + n < L) {
      a = r[(size_t)t * L + n0 + n];
      b = r[(size_t)(nt + t) * L + n0 + n];
    }
    buf[n * nt + bitrev(t, logn)] = make_double2(a, b);
  }
  __syncthreads();
  lds_fft(buf, TN, nt, logn, tw, false);
  const double st = sqrt(tau);
  for (int e = threadIdx.x; e < TN * nf; e += blockDim.x) {
    const int n = e % TN, j = e / TN;
    const int g = n0 + n;
    if (g >= L) continue;
    const double2 Zj = buf[n * nt + j], Zm = buf[n * nt + ((nt - j) & (nt - 1))];
    double2 X0 = make_double2(0.5 * (Zj.x + Zm.x), 0.5 * (Zj.y - Zm.y));
    double2 X1 = make_double2(0.5 * (Zj.y + Zm.y), -0.5 * (Zj.x - Zm.x));
    const bool vel = g < 2 * nq2;
    if (mode == 1) {
      const double dc = tj[j].x, c2 = tj[j].y;
      // s1 = r1/sqrt(tau), s2 = (c2/sqrt(tau)) (r2 - i dc r1/tau)       (velocity)
      // s3 = r3/(sqrt(tau) c2), s4 = (r4 - i dc r3/tau)/sqrt(tau)         (pressure)
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
    if (vel) {
      const int comp = g >= nq2, node = g - comp * nq2;
      V[((size_t)(j * 2 + 0) * 2 + comp) * nq2 + node] = cmk<cpx<R>>(X0.x, X0.y);
      V[((size_t)(j * 2 + 1) * 2 + comp) * nq2 + node] = cmk<cpx<R>>(X1.x, X1.y);
    } else {
      const int node = g - 2 * nq2;
      P[(size_t)(j * 2 + 0) * np2 + node] = cmk<cpx<R>>(X0.x, X0.y);
      P[(size_t)(j * 2 + 1) * np2 + node] = cmk<cpx<R>>(X1.x, X1.y);
    }
  }
}

// Inverse: V, P hold the block solutions x (Stokes: of Z_j; Oseen: of G_j) at
// j = 0..nt/2.  mode 1 applies T_r^{-1} first.  The full spectrum is rebuilt
// from Y_{nt-j} = conj(Y_j), packed as Z_j = Y0_j + i Y1_j, transformed with
// exp(+2 pi i j t / nt) and scaled by 1/nt:  z[b=0] = Re, z[b=1] = Im.
template <typename R>
__global__ __launch_bounds__(256) void k_time_fft_inv(const cpx<R>* __restrict__ V, const cpx<R>* __restrict__ P, double* __restrict__ z,
                               int nt, int logn, int L, int nq2, int np2, int nf, int TN,
                               const double2* __restrict__ tw, const double2* __restrict__ tj, double tau, int mode) {
  extern __shared__ double2 buf[];
  const int n0 = blockIdx.x * TN;
  const double st = sqrt(tau);
  for (int e = threadIdx.x; e < TN * nt; e += blockDim.x) {
    const int n = e % TN, j = e / TN;
    const int g = n0 + n;
    double2 Zv = make_double2(0, 0);
    if (g < L) {
      const bool cj = j > (nt >> 1);
      const int jj = cj ? nt - j : j;
      const bool vel = g < 2 * nq2;
      cpx<R> a, b;
      if (vel) {
        const int comp = g >= nq2, node = g - comp * nq2;
        a = V[((size_t)(jj * 2 + 0) * 2 + comp) * nq2 + node];
        b = V[((size_t)(jj * 2 + 1) * 2 + comp) * nq2 + node];
      } else {
        const int node = g - 2 * nq2;
        a = P[(size_t)(jj * 2 + 0) * np2 + node];
        b = P[(size_t)(jj * 2 + 1) * np2 + node];
      }
      double2 Y0 = make_double2((double)a.x, (double)a.y), Y1 = make_double2((double)b.x, (double)b.y);
      if (mode == 1) {
        const double dc = tj[jj].x, c2 = tj[jj].y;
        if (vel) {
          // y2 = c2 x2 / sqrt(tau);  y1 = (x1 + i dc y2 / sqrt(tau)) / sqrt(tau)
          const double2 y2 = (c2 / st) * Y1;
          const double2 y1 = (1.0 / st) * (Y0 + make_double2(-dc * y2.y / st, dc * y2.x / st));
          Y0 = y1; Y1 = y2;
        } else {
          // y4 = x4 / sqrt(tau);  y3 = (x3 + i dc c2 y4 / sqrt(tau)) / (sqrt(tau) c2)
          const double2 y4 = (1.0 / st) * Y1;
          const double2 y3 = (1.0 / (st * c2)) * (Y0 + make_double2(-dc * c2 * y4.y / st, dc * c2 * y4.x / st));
          Y0 = y3; Y1 = y4;
        }
      }
      if (cj) { Y0.y = -Y0.y; Y1.y = -Y1.y; }
      Zv = make_double2(Y0.x - Y1.y, Y0.y + Y1.x);        // Y0 + i Y1
    }
    buf[n * nt + bitrev(j, logn)] = Zv;
  }
  __syncthreads();
  lds_fft(buf, TN, nt, logn, tw, true);
  const double sc = 1.0 / nt;
  for (int e = threadIdx.x; e < TN * nt; e += blockDim.x) {
    const int n = e % TN, t = e / TN;
    if (n0 + n >= L) continue;
    const double2 v = buf[n * nt + t];
    z[(size_t)t * L + n0 + n] = sc * v.x;
    z[(size_t)(nt + t) * L + n0 + n] = sc * v.y;
  }
}

static int fft_tile(int nt) {
  int tn = 4096 / nt;            // 64 KiB of LDS per work-group
  return tn < 1 ? 1 : (tn > 32 ? 32 : tn);
}

template <typename R>
void launch_time_fft_fwd(hipStream_t s, const double* r, cpx<R>* V, cpx<R>* P, int nt, int L, int nq2, int np2,
                         const double2* tw, const double2* tj, double tau, int mode) {
  int logn = 0;
  while ((1 << logn) < nt) ++logn;
  const int TN = fft_tile(nt), nf = nt / 2 + 1;
  const unsigned blocks = (unsigned)((L + TN - 1) / TN);
  hipLaunchKernelGGL(k_time_fft_fwd<R>, dim3(blocks), dim3(256), (size_t)TN * nt * sizeof(double2), s, r, V, P, nt,
                     logn, L, nq2, np2, nf, TN, tw, tj, tau, mode);
}

template <typename R>
void launch_time_fft_inv(hipStream_t s, const cpx<R>* V, const cpx<R>* P, double* z, int nt, int L, int nq2,
                         int np2, const double2* tw, const double2* tj, double tau, int mode) {
  int logn = 0;
  while ((1 << logn) < nt) ++logn;
  const int TN = fft_tile(nt), nf = nt / 2 + 1;
  const unsigned blocks = (unsigned)((L + TN - 1) / TN);
  hipLaunchKernelGGL(k_time_fft_inv<R>, dim3(blocks), dim3(256), (size_t)TN * nt * sizeof(double2), s, V, P, z, nt,
                     logn, L, nq2, np2, nf, TN, tw, tj, tau, mode);
}

template void launch_time_fft_fwd<double>(hipStream_t, const double*, double2*, double2*, int, int, int, int,
                                          const double2*, const double2*, double, int);
template void launch_time_fft_fwd<float>(hipStream_t, const double*, float2*, float2*, int, int, int, int,
                                         const double2*, const double2*, double, int);
template void launch_time_fft_inv<double>(hipStream_t, const double2*, const double2*, double*, int, int, int, int,
                                          const double2*, const double2*, double, int);
template void launch_time_fft_inv<float>(hipStream_t, const float2*, const float2*, double*, int, int, int, int,
                                         const double2*, const double2*, double, int);

}  // namespace pintoc
