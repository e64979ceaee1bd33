// Kernels of the per-frequency inner solves (Algorithm 2): the Stokes block
// Z_j (section 3.2) applied matrix-free, and the batched complex vector
// operations of one GMRES per frequency.
//
// A "frequency vector" holds, for every kept frequency j, the four fields of
// eq. (SubBlockG) in (v, lambda, p, mu) order:
//   V part [j][b][comp][(2N+1)^2]   b = 0: v,  b = 1: lambda
//   P part [j][b][(N+1)^2]          b = 0: p,  b = 1: mu   (node 0 pinned, zero)
// Dot products are per frequency with the Hermitian inner product, reduced in
// a fixed order (chunk partial sums, then a sequential sum over chunks).
#include "kernels.h"

namespace pintoc {

// ------------------------------------------------------ per-frequency BLAS
// Geometry of a frequency vector: per frequency segV complex entries in the V
// part and segP in the P part; basis vector i starts at i*ldV / i*ldP.
constexpr int kFChunk = 2048;   // entries per work-group and chunk
constexpr int kFK = 16;         // basis vectors per dot pass

template <typename R>
__global__ __launch_bounds__(256) void k_fdot(const cpx<R>* __restrict__ bV, const cpx<R>* __restrict__ bP, size_t ldV, size_t ldP, int k,
                       const cpx<R>* __restrict__ wV, const cpx<R>* __restrict__ wP, int segV, int segP, int chV,
                       int nch, int nf, double2* __restrict__ part, Mask mk) {
  __shared__ double red[2][256];
  const int j = blockIdx.y, c = blockIdx.x;
  if (mk.off(j)) return;
  const bool inV = c < chV;
  const int seg = inV ? segV : segP;
  const int cc = inV ? c : c - chV;
  const size_t base = (size_t)j * seg;
  const cpx<R>* B = inV ? bV : bP;
  const cpx<R>* W = inV ? wV : wP;
  const size_t ld = inV ? ldV : ldP;
  double ar[kFK], ai[kFK];
#pragma unroll
  for (int i = 0; i < kFK; ++i) { ar[i] = 0; ai[i] = 0; }
  const int lo = cc * kFChunk, hi = min(lo + kFChunk, seg);
  for (int e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    const cpx<R> w = W[base + e];
    const double wr = (double)w.x, wi = (double)w.y;
#pragma unroll
    for (int i = 0; i < kFK; ++i) {
      if (i < k) {
        const cpx<R> v = B[i * ld + base + e];
        ar[i] += (double)v.x * wr + (double)v.y * wi;      // conj(v) * w
        ai[i] += (double)v.x * wi - (double)v.y * wr;
      }
    }
  }
  for (int i = 0; i < k; ++i) {
    red[0][threadIdx.x] = ar[i];
    red[1][threadIdx.x] = ai[i];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) {
        red[0][threadIdx.x] += red[0][threadIdx.x + st];
        red[1][threadIdx.x] += red[1][threadIdx.x + st];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((size_t)i * nf + j) * nch + c] = make_double2(red[0][0], red[1][0]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_fdot_reduce(const double2* __restrict__ part, int k, int nf, int nch, double2* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * nf) return;
  double sr = 0, si = 0;
  for (int c = 0; c < nch; ++c) { const double2 v = part[(size_t)t * nch + c]; sr += v.x; si += v.y; }
  out[t] = make_double2(sr, si);
}

// w^j -= sum_i c[i][j] v_i^j    (c: [k][nf] complex, on the device)
template <typename R>
__global__ __launch_bounds__(256) void k_fupdate(cpx<R>* __restrict__ wV, cpx<R>* __restrict__ wP, const cpx<R>* __restrict__ bV,
                          const cpx<R>* __restrict__ bP, size_t ldV, size_t ldP, int k, const double2* __restrict__ c,
                          int segV, int segP, int nf, double sign, Mask mk) {
  const int j = blockIdx.y;
  if (mk.off(j)) return;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool inV = e < (size_t)segV;
  if (!inV && e >= (size_t)segV + segP) return;
  const size_t off = inV ? (size_t)j * segV + e : (size_t)j * segP + (e - segV);
  cpx<R>* W = inV ? wV : wP;
  const cpx<R>* B = inV ? bV : bP;
  const size_t ld = inV ? ldV : ldP;
  double sr = 0, si = 0;
  for (int i = 0; i < k; ++i) {
    const double2 ci = c[(size_t)i * nf + j];
    const cpx<R> v = B[i * ld + off];
    sr += ci.x * (double)v.x - ci.y * (double)v.y;
    si += ci.x * (double)v.y + ci.y * (double)v.x;
  }
  cpx<R> w = W[off];
  W[off] = cmk<cpx<R>>((double)w.x - sign * sr, (double)w.y - sign * si);
}

// y^j = a[j] x^j   (a complex per frequency; y may alias x)
template <typename R>
__global__ __launch_bounds__(256) void k_fscale(cpx<R>* yV, cpx<R>* yP, const cpx<R>* xV, const cpx<R>* xP, const double2* __restrict__ a,
                         int segV, int segP, Mask mk) {
  const int j = blockIdx.y;
  if (mk.off(j)) return;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool inV = e < (size_t)segV;
  if (!inV && e >= (size_t)segV + segP) return;
  const size_t off = inV ? (size_t)j * segV + e : (size_t)j * segP + (e - segV);
  const cpx<R> x = inV ? xV[off] : xP[off];
  const double2 s = a[j];
  const cpx<R> y = cmk<cpx<R>>(s.x * (double)x.x - s.y * (double)x.y, s.x * (double)x.y + s.y * (double)x.x);
  if (inV) yV[off] = y; else yP[off] = y;
}

// unpinned copy of the pressure fields: dst = src with dst[f][0] = -sum_{i>=1} src[f][i]
template <typename R>
__global__ __launch_bounds__(256) void k_unpin_copy(cpx<R>* __restrict__ dst, const cpx<R>* __restrict__ src, int nn, Mask mk) {
  __shared__ double sr[256], si[256];
  const int f = blockIdx.x;
  if (mk.off(f)) return;
  const cpx<R>* g = src + (size_t)f * nn;
  cpx<R>* d = dst + (size_t)f * nn;
  double ar = 0, ai = 0;
  for (int i = 1 + threadIdx.x; i < nn; i += blockDim.x) {
    const cpx<R> v = g[i];
    ar += (double)v.x; ai += (double)v.y;
    d[i] = v;
  }
  sr[threadIdx.x] = ar; si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; si[threadIdx.x] += si[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) d[0] = cmk<cpx<R>>(-sr[0], -si[0]);
}

// (de)conversion between the FP64 FFT output and a precision-R frequency vector
template <typename Rd, typename Rs>
__global__ __launch_bounds__(256) void k_convert(cpx<Rd>* __restrict__ d, const cpx<Rs>* __restrict__ s, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const cpx<Rs> v = s[e];
    d[e] = cmk<cpx<Rd>>((double)v.x, (double)v.y);
  }
}

template <typename R>
void launch_fdot(hipStream_t s, const cpx<R>* bV, const cpx<R>* bP, size_t ldV, size_t ldP, int k, const cpx<R>* wV,
                 const cpx<R>* wP, int segV, int segP, int nf, double2* part, double2* out, Mask mk) {
  const int chV = (segV + kFChunk - 1) / kFChunk, chP = (segP + kFChunk - 1) / kFChunk, nch = chV + chP;
  for (int i0 = 0; i0 < k; i0 += kFK) {
    const int kk = k - i0 < kFK ? k - i0 : kFK;
    hipLaunchKernelGGL(k_fdot<R>, dim3(nch, nf), dim3(256), 0, s, bV + i0 * ldV, bP + i0 * ldP, ldV, ldP, kk, wV, wP,
                       segV, segP, chV, nch, nf, part, mk);
    hipLaunchKernelGGL(k_fdot_reduce, dim3((kk * nf + 255) / 256), dim3(256), 0, s, part, kk, nf, nch,
                       out + (size_t)i0 * nf);
  }
}

size_t fdot_part_entries(int segV, int segP, int nf) {
  const int nch = (segV + kFChunk - 1) / kFChunk + (segP + kFChunk - 1) / kFChunk;
  return (size_t)kFK * nf * nch;
}

template <typename R>
void launch_fupdate(hipStream_t s, cpx<R>* wV, cpx<R>* wP, const cpx<R>* bV, const cpx<R>* bP, size_t ldV,
                    size_t ldP, int k, const double2* c, int segV, int segP, int nf, double sign, Mask mk) {
  const size_t tot = (size_t)segV + segP;
  hipLaunchKernelGGL(k_fupdate<R>, dim3((unsigned)((tot + 255) / 256), nf), dim3(256), 0, s, wV, wP, bV, bP, ldV,
                     ldP, k, c, segV, segP, nf, sign, mk);
}

template <typename R>
void launch_fscale(hipStream_t s, cpx<R>* yV, cpx<R>* yP, const cpx<R>* xV, const cpx<R>* xP, const double2* a,
                   int segV, int segP, int nf, Mask mk) {
  const size_t tot = (size_t)segV + segP;
  hipLaunchKernelGGL(k_fscale<R>, dim3((unsigned)((tot + 255) / 256), nf), dim3(256), 0, s, yV, yP, xV, xP, a, segV,
                     segP, mk);
}

template <typename R>
void launch_unpin_copy(hipStream_t s, cpx<R>* dst, const cpx<R>* src, int nn, int nb, Mask mk) {
  hipLaunchKernelGGL(k_unpin_copy<R>, dim3(nb), dim3(256), 0, s, dst, src, nn, mk);
}

template <typename Rd, typename Rs>
void launch_convert(hipStream_t s, cpx<Rd>* d, const cpx<Rs>* src, size_t n) {
  hipLaunchKernelGGL((k_convert<Rd, Rs>), dim3(2048), dim3(256), 0, s, d, src, n);
}

#define PINTOC_INNER_INST(R)                                                                                       \
  template void launch_fdot<R>(hipStream_t, const cpx<R>*, const cpx<R>*, size_t, size_t, int, const cpx<R>*,      \
                               const cpx<R>*, int, int, int, double2*, double2*, Mask);                                  \
  template void launch_fupdate<R>(hipStream_t, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*, size_t, size_t, int, \
                                  const double2*, int, int, int, double, Mask);                                          \
  template void launch_fscale<R>(hipStream_t, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*, const double2*, int, \
                                 int, int, Mask);                                                                        \
  template void launch_unpin_copy<R>(hipStream_t, cpx<R>*, const cpx<R>*, int, int, Mask);

PINTOC_INNER_INST(double)
PINTOC_INNER_INST(float)
template void launch_convert<double, float>(hipStream_t, double2*, const float2*, size_t);
template void launch_convert<float, double>(hipStream_t, float2*, const double2*, size_t);

}  // namespace pintoc
