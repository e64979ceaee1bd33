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
// A work-group takes a tile [t = 0..nt-1] x [16 consecutive n] (coalesced along
// n) and writes [j][16 consecutive n] (coalesced along n).  For nt <= 256 the
// transform is the four-step split nt = N1 N2 with both factor transforms in
// registers and two LDS exchanges; longer sequences use radix-2 stages in LDS
// over 4096/nt level indices per work-group.
//
// Frequency-domain layout:  V[j][b][comp][(2N+1)^2], P[j][b][(N+1)^2] (complex).
#include "kernels.h"

namespace pintoc {

__device__ inline int bitrev(int v, int logn) { return (int)(__brev((unsigned)v) >> (32 - logn)); }

// Tile of a work-group (or ~0u past the last of ntile tiles).  Work-group ids
// are dealt round-robin to the 8 XCDs, so id g takes tile (g % 8) (G / 8) +
// g / 8 (G, the grid, a multiple of 8): each XCD runs a contiguous range of
// level indices, and the cache lines that two neighbouring tiles share (rows
// of L or (2N+1)^2 entries start at any offset) meet in one L2.
__device__ __forceinline__ unsigned xcd_tile(int ntile) {
  const unsigned v = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  return v < (unsigned)ntile ? v : ~0u;
}
__host__ inline unsigned xcd_grid(int ntile) { return (unsigned)((ntile + 7) / 8 * 8); }

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
  const unsigned tile = xcd_tile((L + TN - 1) / TN);
  if (tile == ~0u) return;
  const int n0 = (int)tile * TN;
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
  const unsigned tile = xcd_tile((L + TN - 1) / TN);
  if (tile == ~0u) return;
  const int n0 = (int)tile * TN;
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

// ---- four-step transform, nt = N1 N2 <= 256 ------------------------------
// With t = N2 t1 + t2 and k = k1 + N1 k2 the length-nt DFT factors as
//   X[k1 + N1 k2] = sum_t2 W_N2^(t2 k2) W_nt^(t2 k1) sum_t1 x[N2 t1 + t2] W_N1^(t1 k1),
// W_m = exp(-+2 pi i / m).  A work-group of 16 N1 threads holds 16 level
// indices; thread (n, c), n = threadIdx.x mod 16, c = threadIdx.x / 16, runs
// the length-N1 transform of column t2 = c (if c < N2) and then the length-N2
// transform of row k1 = c.  LDS keeps element p of level index n at
// p * 16 + n, so lane j of every 16-lane group sits on 16-byte residue j in
// all accesses (conflict-free 128-bit LDS reads and writes).
constexpr int kFN = 16;

// v * exp(-+2 pi i q / 16), q in [0, 8): cos and sin of multiples of pi / 8.
__device__ __forceinline__ double2 rot16(double2 v, int q, bool inv) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
  double c, sn;
  switch (q) {
    case 0: return v;
    case 4: return inv ? make_double2(-v.y, v.x) : make_double2(v.y, -v.x);
    case 1: c = c1; sn = s1; break;
    case 2: c = h; sn = h; break;
    case 3: c = s1; sn = c1; break;
    case 5: c = -s1; sn = c1; break;
    case 6: c = -h; sn = h; break;
    default: c = -c1; sn = s1; break;
  }
  if (!inv) sn = -sn;
  return make_double2(v.x * c - v.y * sn, v.x * sn + v.y * c);
}

template <int M> __host__ __device__ constexpr int brev_c(int i) {
  int r = 0;
  for (int b = 1; b < M; b <<= 1) { r = (r << 1) | (i & 1); i >>= 1; }
  return r;
}

// In-register length-M DFT (M in {1, 2, 4, 8, 16}), natural order in and out:
// bit-reversal permutation, then radix-2 decimation-in-time stages.
template <int M, bool INV>
__device__ __forceinline__ void reg_fft(double2 (&x)[M]) {
  double2 y[M];
#pragma unroll
  for (int i = 0; i < M; ++i) y[brev_c<M>(i)] = x[i];
#pragma unroll
  for (int m = 1; m < M; m <<= 1) {
#pragma unroll
    for (int i0 = 0; i0 < M; i0 += 2 * m) {
#pragma unroll
      for (int q = 0; q < m; ++q) {
        const double2 a = y[i0 + q], b = rot16(y[i0 + q + m], q * (16 / (2 * m)), INV);
        y[i0 + q] = a + b;
        y[i0 + q + m] = a - b;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < M; ++i) x[i] = y[i];
}

// exp(-+2 pi i e / nt) for 0 <= e < nt from the half table tw[k] = exp(-2 pi i k / nt).
__device__ __forceinline__ double2 tw_at(const double2* __restrict__ tw, int e, int nt, bool inv) {
  const int h = nt >> 1;
  double2 w = tw[e & (h - 1)];
  if (e & h) { w.x = -w.x; w.y = -w.y; }
  if (inv) w.y = -w.y;
  return w;
}

template <typename R, int N1, int N2>
__global__ __launch_bounds__(kFN * N1) void k_fft4_fwd(const double* __restrict__ r, cpx<R>* __restrict__ V,
                                                       cpx<R>* __restrict__ P, int L, int nq2, int np2,
                                                       const double2* __restrict__ tw, const double2* __restrict__ tj,
                                                       double tau, int mode) {
  constexpr int NT = N1 * N2, NF = NT / 2 + 1;
  __shared__ double2 buf[NT * kFN];
  const int n = threadIdx.x & (kFN - 1), c = threadIdx.x / kFN;
  const unsigned tile = xcd_tile((L + kFN - 1) / kFN);
  if (tile == ~0u) return;
  const int n0 = (int)tile * kFN, g = n0 + n;
  const bool live = g < L;
  if (c < N2) {                                   // pass 1: column t2 = c
    double2 x[N1];
#pragma unroll
    for (int t1 = 0; t1 < N1; ++t1) {
      const size_t t = (size_t)(N2 * t1 + c);
      x[t1] = live ? make_double2(r[t * L + g], r[(NT + t) * L + g]) : make_double2(0.0, 0.0);
    }
    reg_fft<N1, false>(x);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1)
      buf[(N2 * k1 + c) * kFN + n] = k1 == 0 ? x[0] : cmul(x[k1], tw_at(tw, c * k1, NT, false));
  }
  __syncthreads();
  {                                               // pass 2: row k1 = c; X[c + N1 k2] kept at N2 c + k2
    double2 x[N2];
#pragma unroll
    for (int t2 = 0; t2 < N2; ++t2) x[t2] = buf[(N2 * c + t2) * kFN + n];
    reg_fft<N2, false>(x);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) buf[(N2 * c + k2) * kFN + n] = x[k2];
  }
  __syncthreads();
  if (!live) return;
  const double st = sqrt(tau);
  for (int j = c; j < NF; j += N1) {
    const int jm = (NT - j) & (NT - 1);
    const double2 Zj = buf[(N2 * (j % N1) + j / N1) * kFN + n];
    const double2 Zm = buf[(N2 * (jm % N1) + jm / N1) * kFN + n];
    double2 X0 = make_double2(0.5 * (Zj.x + Zm.x), 0.5 * (Zj.y - Zm.y));
    double2 X1 = make_double2(0.5 * (Zj.y + Zm.y), -0.5 * (Zj.x - Zm.x));
    const bool vel = g < 2 * nq2;
    if (mode == 1) {
      const double dc = tj[j].x, c2 = tj[j].y;
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

template <typename R, int N1, int N2>
__global__ __launch_bounds__(kFN * N1) void k_fft4_inv(const cpx<R>* __restrict__ V, const cpx<R>* __restrict__ P,
                                                       double* __restrict__ z, int L, int nq2, int np2,
                                                       const double2* __restrict__ tw, const double2* __restrict__ tj,
                                                       double tau, int mode) {
  constexpr int NT = N1 * N2, NF = NT / 2 + 1;
  __shared__ double2 buf[NT * kFN];
  const int n = threadIdx.x & (kFN - 1), c = threadIdx.x / kFN;
  const unsigned tile = xcd_tile((L + kFN - 1) / kFN);
  if (tile == ~0u) return;
  const int g = (int)tile * kFN + n;
  const bool live = g < L;
  const double st = sqrt(tau);
  // Spectrum of z = y0 + i y1 at j and nt - j from the kept j = 0..nt/2.
#pragma unroll
  for (int i = 0; i < (NF + N1 - 1) / N1; ++i) {
    const int jj = c + i * N1;
    if (jj >= NF) break;
    double2 Zv = make_double2(0.0, 0.0), Zc = Zv;
    if (live) {
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
          const double2 y2 = (c2 / st) * Y1;
          const double2 y1 = (1.0 / st) * (Y0 + make_double2(-dc * y2.y / st, dc * y2.x / st));
          Y0 = y1; Y1 = y2;
        } else {
          const double2 y4 = (1.0 / st) * Y1;
          const double2 y3 = (1.0 / (st * c2)) * (Y0 + make_double2(-dc * c2 * y4.y / st, dc * c2 * y4.x / st));
          Y0 = y3; Y1 = y4;
        }
      }
      Zv = make_double2(Y0.x - Y1.y, Y0.y + Y1.x);          // Y0 + i Y1
      Zc = make_double2(Y0.x + Y1.y, Y1.x - Y0.y);          // conj(Y0) + i conj(Y1)
    }
    buf[jj * kFN + n] = Zv;
    if (jj > 0 && jj < NT / 2) buf[(NT - jj) * kFN + n] = Zc;
  }
  __syncthreads();
  if (c < N2) {                                   // pass 1: column t2 = c, in place
    double2 x[N1];
#pragma unroll
    for (int t1 = 0; t1 < N1; ++t1) x[t1] = buf[(N2 * t1 + c) * kFN + n];
    reg_fft<N1, true>(x);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1)
      buf[(N2 * k1 + c) * kFN + n] = k1 == 0 ? x[0] : cmul(x[k1], tw_at(tw, c * k1, NT, true));
  }
  __syncthreads();
  if (!live) return;
  double2 x[N2];                                  // pass 2: row k1 = c -> t = c + N1 k2
#pragma unroll
  for (int t2 = 0; t2 < N2; ++t2) x[t2] = buf[(N2 * c + t2) * kFN + n];
  reg_fft<N2, true>(x);
  const double sc = 1.0 / NT;
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) {
    const size_t t = (size_t)(c + N1 * k2);
    z[t * L + g] = sc * x[k2].x;
    z[(NT + t) * L + g] = sc * x[k2].y;
  }
}

template <typename R, int N1, int N2>
static void fft4_fwd(hipStream_t s, const double* r, cpx<R>* V, cpx<R>* P, int L, int nq2, int np2,
                     const double2* tw, const double2* tj, double tau, int mode) {
  hipLaunchKernelGGL((k_fft4_fwd<R, N1, N2>), dim3(xcd_grid((L + kFN - 1) / kFN)), dim3(kFN * N1), 0, s, r, V, P, L,
                     nq2, np2, tw, tj, tau, mode);
}

template <typename R, int N1, int N2>
static void fft4_inv(hipStream_t s, const cpx<R>* V, const cpx<R>* P, double* z, int L, int nq2, int np2,
                     const double2* tw, const double2* tj, double tau, int mode) {
  hipLaunchKernelGGL((k_fft4_inv<R, N1, N2>), dim3(xcd_grid((L + kFN - 1) / kFN)), dim3(kFN * N1), 0, s, V, P, z, L,
                     nq2, np2, tw, tj, tau, mode);
}

static int fft_tile(int nt) {
  int tn = 4096 / nt;            // 64 KiB of LDS per work-group
  return tn < 1 ? 1 : (tn > 32 ? 32 : tn);
}

template <typename R>
void launch_time_fft_fwd(hipStream_t s, const double* r, cpx<R>* V, cpx<R>* P, int nt, int L, int nq2, int np2,
                         const double2* tw, const double2* tj, double tau, int mode) {
  switch (nt) {
    case 2: return fft4_fwd<R, 2, 1>(s, r, V, P, L, nq2, np2, tw, tj, tau, mode);
    case 4: return fft4_fwd<R, 2, 2>(s, r, V, P, L, nq2, np2, tw, tj, tau, mode);
    case 8: return fft4_fwd<R, 4, 2>(s, r, V, P, L, nq2, np2, tw, tj, tau, mode);
    case 16: return fft4_fwd<R, 4, 4>(s, r, V, P, L, nq2, np2, tw, tj, tau, mode);
    case 32: return fft4_fwd<R, 8, 4>(s, r, V, P, L, nq2, np2, tw, tj, tau, mode);
    case 64: return fft4_fwd<R, 8, 8>(s, r, V, P, L, nq2, np2, tw, tj, tau, mode);
    case 128: return fft4_fwd<R, 16, 8>(s, r, V, P, L, nq2, np2, tw, tj, tau, mode);
    case 256: return fft4_fwd<R, 16, 16>(s, r, V, P, L, nq2, np2, tw, tj, tau, mode);
    default: break;
  }
  int logn = 0;
  while ((1 << logn) < nt) ++logn;
  const int TN = fft_tile(nt), nf = nt / 2 + 1;
  const unsigned blocks = xcd_grid((L + TN - 1) / TN);
  hipLaunchKernelGGL(k_time_fft_fwd<R>, dim3(blocks), dim3(256), (size_t)TN * nt * sizeof(double2), s, r, V, P, nt,
                     logn, L, nq2, np2, nf, TN, tw, tj, tau, mode);
}

template <typename R>
void launch_time_fft_inv(hipStream_t s, const cpx<R>* V, const cpx<R>* P, double* z, int nt, int L, int nq2,
                         int np2, const double2* tw, const double2* tj, double tau, int mode) {
  switch (nt) {
    case 2: return fft4_inv<R, 2, 1>(s, V, P, z, L, nq2, np2, tw, tj, tau, mode);
    case 4: return fft4_inv<R, 2, 2>(s, V, P, z, L, nq2, np2, tw, tj, tau, mode);
    case 8: return fft4_inv<R, 4, 2>(s, V, P, z, L, nq2, np2, tw, tj, tau, mode);
    case 16: return fft4_inv<R, 4, 4>(s, V, P, z, L, nq2, np2, tw, tj, tau, mode);
    case 32: return fft4_inv<R, 8, 4>(s, V, P, z, L, nq2, np2, tw, tj, tau, mode);
    case 64: return fft4_inv<R, 8, 8>(s, V, P, z, L, nq2, np2, tw, tj, tau, mode);
    case 128: return fft4_inv<R, 16, 8>(s, V, P, z, L, nq2, np2, tw, tj, tau, mode);
    case 256: return fft4_inv<R, 16, 16>(s, V, P, z, L, nq2, np2, tw, tj, tau, mode);
    default: break;
  }
  int logn = 0;
  while ((1 << logn) < nt) ++logn;
  const int TN = fft_tile(nt), nf = nt / 2 + 1;
  const unsigned blocks = xcd_grid((L + TN - 1) / TN);
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
