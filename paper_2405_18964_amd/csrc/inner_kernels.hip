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
#include <algorithm>

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
  // sequential sum in chunk order; the unrolled loads are issued ahead of the adds
  double sr = 0, si = 0;
  const double2* pt = part + (size_t)t * nch;
  int c = 0;
  for (; c + 8 <= nch; c += 8) {
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = pt[c + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) { sr += v[q].x; si += v[q].y; }
  }
  for (; c < nch; ++c) { const double2 v = pt[c]; sr += v.x; si += v.y; }
  out[t] = make_double2(sr, si);
}

// ---------------------------------------------- lagged reorthogonalisation
// Arnoldi with classical Gram-Schmidt applied twice, where the second pass of
// one column is carried out together with the first pass of the next (the
// matrix acts on the once-projected vector u_k; the host corrects the
// Hessenberg column through the Arnoldi relation).  Per iteration the basis is
// read twice: one fused dot pass and one fused update pass.
//
// Dot pass, per frequency: s_i = q_i^H u, t_i = q_i^H w (i < k), nu = u^H u,
// mu = u^H w, with q_i = basis vector i, u = basis vector k, w = basis vector
// k + 1 (w == nullptr: s and nu only).  One launch covers i in [i0, i1) (nu
// and mu with i0 = 0); wave q of a work-group handles i = i0 + q, i0 + q + 8,
// ...; partial sums per chunk go to
// part[(slot * nf + j) * nch + chunk], slots s_0..s_{k-1}, t_0..t_{k-1}, nu, mu.
constexpr int kLW = 7;                   // basis vectors per wave
constexpr int kLWaves = 6;               // waves per work-group: k <= 42 per launch

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// kU consecutive complex entries at p (16-byte loads: one FP64 or two FP32 entries)
template <typename R, int kU> struct Pack;
template <> struct Pack<double, 1> {
  double2 v[1];
  __device__ __forceinline__ void load(const double2* p) { v[0] = *p; }
  __device__ __forceinline__ void zero() { v[0] = make_double2(0, 0); }
};
template <> struct Pack<float, 2> {
  float2 v[2];
  __device__ __forceinline__ void load(const float2* p) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = make_float2(q.x, q.y);
    v[1] = make_float2(q.z, q.w);
  }
  __device__ __forceinline__ void zero() { v[0] = make_float2(0, 0); v[1] = v[0]; }
};

// Work-groups of 64 W threads (W = blockDim.x / 64 waves); wave q takes the
// basis vectors i = i0 + q + W r.  Every lane reads 16 bytes per vector and
// step (one FP64 or two FP32 entries); segments and chunk bounds are even.
template <typename R>
__global__ __launch_bounds__(64 * kLWaves) void k_fdot_lag(const cpx<R>* __restrict__ bV, const cpx<R>* __restrict__ bP,
                                                  size_t ldV, size_t ldP, int k, int i0, int i1,
                                                  const cpx<R>* __restrict__ uV,
                                                  const cpx<R>* __restrict__ uP, const cpx<R>* __restrict__ wV,
                                                  const cpx<R>* __restrict__ wP, int segV, int segP, int chV, int nch,
                                                  int nf, double2* __restrict__ part, Mask mk) {
  constexpr int kU = sizeof(R) == 4 ? 2 : 1;
  const int j = blockIdx.y, c = blockIdx.x;
  if (mk.off(j)) return;
  const bool inV = c < chV;
  const int seg = inV ? segV : segP;
  const int cc = inV ? c : c - chV;
  const size_t base = (size_t)j * seg;
  const cpx<R>* B = inV ? bV : bP;
  const cpx<R>* U = inV ? uV : uP;
  const cpx<R>* W = inV ? wV : wP;
  const size_t ld = inV ? ldV : ldP;
  const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool mine = wv == 0 && i0 == 0;          // this wave also forms nu and mu
  bool any = mine;
#pragma unroll
  for (int q = 0; q < kLW; ++q) any |= i0 + wv + nw * q < i1;
  // per-lane partial sums in the storage precision (a lane adds at most
  // kFChunk / 64 products), the wave and chunk reductions in FP64
  R sr[kLW], si[kLW], tr[kLW], ti[kLW];
#pragma unroll
  for (int q = 0; q < kLW; ++q) { sr[q] = 0; si[q] = 0; tr[q] = 0; ti[q] = 0; }
  R nu = 0, mur = 0, mui = 0;
  const int lo = cc * kFChunk, hi = min(lo + kFChunk, seg);
  for (int e = lo + kU * lane; any && e < hi; e += 64 * kU) {
    Pack<R, kU> u, w;
    u.load(U + base + e);
    if (W) w.load(W + base + e);
    else w.zero();
    Pack<R, kU> vv[kLW];
#pragma unroll
    for (int q = 0; q < kLW; ++q) {
      const int i = i0 + wv + nw * q;
      if (i < i1) vv[q].load(B + (size_t)i * ld + base + e);
      else vv[q].zero();
    }
#pragma unroll
    for (int h = 0; h < kU; ++h) {
      const R ur = u.v[h].x, ui = u.v[h].y, wr = w.v[h].x, wi = w.v[h].y;
      if (mine) {
        nu += ur * ur + ui * ui;
        mur += ur * wr + ui * wi;              // conj(u) w
        mui += ur * wi - ui * wr;
      }
#pragma unroll
      for (int q = 0; q < kLW; ++q) {
        const R vr = vv[q].v[h].x, vi = vv[q].v[h].y;
        sr[q] += vr * ur + vi * ui;  si[q] += vr * ui - vi * ur;      // conj(v) u
        tr[q] += vr * wr + vi * wi;  ti[q] += vr * wi - vi * wr;      // conj(v) w
      }
    }
  }
  auto put = [&](int slot, double re, double im) {
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) part[((size_t)slot * nf + j) * nch + c] = make_double2(re, im);
  };
#pragma unroll
  for (int q = 0; q < kLW; ++q) {
    const int i = i0 + wv + nw * q;
    if (i < i1) {
      put(i, sr[q], si[q]);
      if (W) put(k + i, tr[q], ti[q]);
    }
  }
  if (mine) {
    put(2 * k, nu, 0.0);
    if (W) put(2 * k + 1, mur, mui);
  }
}

// Update pass, per frequency j with alpha = ag[j].x, gamma = ag[nf + j]:
//   q_k     = (u - sum_i s_i q_i) / alpha                  (written over u)
//   u_{k+1} = (w - gamma u - sum_i c_i q_i) / alpha        (written over w)
// with s_i = cs[i * nf + j], c_i = cc[i * nf + j], and ||u_{k+1}||^2 partial
// sums per chunk in part[j * nch + chunk].  k = 0: q_0 = u is kept.
template <typename R>
__global__ __launch_bounds__(256) void k_fupdate_lag(cpx<R>* __restrict__ bV, cpx<R>* __restrict__ bP, size_t ldV,
                                                     size_t ldP, int k, const double2* __restrict__ cs,
                                                     const double2* __restrict__ cc, const double2* __restrict__ ag,
                                                     int segV, int segP, int chV, int nch, int nf,
                                                     double2* __restrict__ part, Mask mk) {
  __shared__ double red[4];
  const int j = blockIdx.y, c = blockIdx.x;
  if (mk.off(j)) return;
  const bool inV = c < chV;
  const int seg = inV ? segV : segP;
  const int ch = inV ? c : c - chV;
  const size_t base = (size_t)j * seg;
  cpx<R>* B = inV ? bV : bP;
  const size_t ld = inV ? ldV : ldP;
  const double alpha = ag[j].x, ia = 1.0 / alpha;
  const double2 gam = ag[nf + j];
  cpx<R>* U = B + (size_t)k * ld + base;
  cpx<R>* W = B + (size_t)(k + 1) * ld + base;
  double nrm = 0;
  const int lo = ch * kFChunk, hi = min(lo + kFChunk, seg);
  for (int e0 = lo + (int)threadIdx.x; e0 < hi; e0 += 512) {
    const int e1 = e0 + 256;
    const bool ok1 = e1 < hi;
    const cpx<R> u0 = U[e0], w0 = W[e0];
    const cpx<R> u1 = ok1 ? U[e1] : cmk<cpx<R>>(0, 0), w1 = ok1 ? W[e1] : cmk<cpx<R>>(0, 0);
    double as[2][2] = {{0, 0}, {0, 0}}, ac[2][2] = {{0, 0}, {0, 0}};
#pragma unroll 4
    for (int i = 0; i < k; ++i) {
      const double2 si = cs[(size_t)i * nf + j], ci = cc[(size_t)i * nf + j];
      const cpx<R>* qi = B + (size_t)i * ld + base;
      const cpx<R> v0 = qi[e0], v1 = ok1 ? qi[e1] : cmk<cpx<R>>(0, 0);
      const double v0r = (double)v0.x, v0i = (double)v0.y, v1r = (double)v1.x, v1i = (double)v1.y;
      as[0][0] += si.x * v0r - si.y * v0i;  as[0][1] += si.x * v0i + si.y * v0r;
      ac[0][0] += ci.x * v0r - ci.y * v0i;  ac[0][1] += ci.x * v0i + ci.y * v0r;
      as[1][0] += si.x * v1r - si.y * v1i;  as[1][1] += si.x * v1i + si.y * v1r;
      ac[1][0] += ci.x * v1r - ci.y * v1i;  ac[1][1] += ci.x * v1i + ci.y * v1r;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !ok1) break;
      const int e = h ? e1 : e0;
      const cpx<R> u = h ? u1 : u0, w = h ? w1 : w0;
      const double ur = (double)u.x, ui = (double)u.y;
      if (k > 0) U[e] = cmk<cpx<R>>((ur - as[h][0]) * ia, (ui - as[h][1]) * ia);
      const cpx<R> un = cmk<cpx<R>>(((double)w.x - (gam.x * ur - gam.y * ui) - ac[h][0]) * ia,
                                    ((double)w.y - (gam.x * ui + gam.y * ur) - ac[h][1]) * ia);
      W[e] = un;
      nrm += (double)un.x * (double)un.x + (double)un.y * (double)un.y;
    }
  }
  nrm = wave_sum(nrm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)j * nch + c] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
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

// y = a_j y + b_j x1 + c_j x2 per frequency j with real coefficients
// coef[j], coef[nf + j], coef[2 nf + j] (the three-term updates of the inner
// MINRES); x2 may be null (c_j ignored)
template <typename R>
__global__ __launch_bounds__(256) void k_fcomb3(cpx<R>* __restrict__ yV, cpx<R>* __restrict__ yP,
                                                const cpx<R>* __restrict__ x1V, const cpx<R>* __restrict__ x1P,
                                                const cpx<R>* __restrict__ x2V, const cpx<R>* __restrict__ x2P,
                                                const double* __restrict__ coef, int segV, int segP, int nf,
                                                Mask mk) {
  const int j = blockIdx.y;
  if (mk.off(j)) return;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool inV = e < (size_t)segV;
  if (!inV && e >= (size_t)segV + segP) return;
  const size_t off = inV ? (size_t)j * segV + e : (size_t)j * segP + (e - segV);
  cpx<R>* Y = inV ? yV : yP;
  const cpx<R>* X1 = inV ? x1V : x1P;
  const cpx<R>* X2 = inV ? x2V : x2P;
  const double a = coef[j], b = coef[nf + j];
  const cpx<R> y = Y[off], u = X1[off];
  double re = a * (double)y.x + b * (double)u.x, im = a * (double)y.y + b * (double)u.y;
  if (X2) {
    const double c = coef[2 * nf + j];
    const cpx<R> v = X2[off];
    re += c * (double)v.x;
    im += c * (double)v.y;
  }
  Y[off] = cmk<cpx<R>>(re, im);
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
void launch_fdot_lag(hipStream_t s, const cpx<R>* bV, const cpx<R>* bP, size_t ldV, size_t ldP, int k,
                     const cpx<R>* uV, const cpx<R>* uP, const cpx<R>* wV, const cpx<R>* wP, int segV, int segP,
                     int nf, double2* part, double2* out, Mask mk) {
  const int chV = (segV + kFChunk - 1) / kFChunk, chP = (segP + kFChunk - 1) / kFChunk, nch = chV + chP;
  for (int i0 = 0; i0 < (k > 0 ? k : 1); i0 += kLWaves * kLW) {
    const int i1 = i0 + kLWaves * kLW < k ? i0 + kLWaves * kLW : k;
    const int waves = std::max(1, std::min(kLWaves, (i1 - i0 + kLW - 1) / kLW));
    hipLaunchKernelGGL(k_fdot_lag<R>, dim3(nch, nf), dim3(64 * waves), 0, s, bV, bP, ldV, ldP, k, i0, i1, uV, uP, wV, wP,
                       segV, segP, chV, nch, nf, part, mk);
  }
  const int slots = 2 * k + 2;
  hipLaunchKernelGGL(k_fdot_reduce, dim3((slots * nf + 255) / 256), dim3(256), 0, s, part, slots, nf, nch, out);
}

template <typename R>
void launch_fupdate_lag(hipStream_t s, cpx<R>* bV, cpx<R>* bP, size_t ldV, size_t ldP, int k, const double2* cs,
                        const double2* cc, const double2* ag, int segV, int segP, int nf, double2* part,
                        double2* out, Mask mk) {
  const int chV = (segV + kFChunk - 1) / kFChunk, chP = (segP + kFChunk - 1) / kFChunk, nch = chV + chP;
  hipLaunchKernelGGL(k_fupdate_lag<R>, dim3(nch, nf), dim3(256), 0, s, bV, bP, ldV, ldP, k, cs, cc, ag, segV, segP,
                     chV, nch, nf, part, mk);
  hipLaunchKernelGGL(k_fdot_reduce, dim3((nf + 255) / 256), dim3(256), 0, s, part, 1, nf, nch, out);
}

size_t lag_part_entries(int segV, int segP, int nf, int m) {
  const int nch = (segV + kFChunk - 1) / kFChunk + (segP + kFChunk - 1) / kFChunk;
  return (size_t)(2 * m + 2) * nf * nch;
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
void launch_fcomb3(hipStream_t s, cpx<R>* yV, cpx<R>* yP, const cpx<R>* x1V, const cpx<R>* x1P, const cpx<R>* x2V,
                   const cpx<R>* x2P, const double* coef, int segV, int segP, int nf, Mask mk) {
  const size_t tot = (size_t)segV + segP;
  hipLaunchKernelGGL(k_fcomb3<R>, dim3((unsigned)((tot + 255) / 256), nf), dim3(256), 0, s, yV, yP, x1V, x1P, x2V,
                     x2P, coef, segV, segP, nf, mk);
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
  template void launch_unpin_copy<R>(hipStream_t, cpx<R>*, const cpx<R>*, int, int, Mask);                         \
  template void launch_fcomb3<R>(hipStream_t, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*,       \
                                 const cpx<R>*, const double*, int, int, int, Mask);                               \
  template void launch_fdot_lag<R>(hipStream_t, const cpx<R>*, const cpx<R>*, size_t, size_t, int, const cpx<R>*,  \
                                   const cpx<R>*, const cpx<R>*, const cpx<R>*, int, int, int, double2*, double2*, Mask); \
  template void launch_fupdate_lag<R>(hipStream_t, cpx<R>*, cpx<R>*, size_t, size_t, int, const double2*,           \
                                      const double2*, const double2*, int, int, int, double2*, double2*, Mask);

PINTOC_INNER_INST(double)
PINTOC_INNER_INST(float)
template void launch_convert<double, float>(hipStream_t, double2*, const float2*, size_t);
template void launch_convert<float, double>(hipStream_t, float2*, const double2*, size_t);

}  // namespace pintoc
