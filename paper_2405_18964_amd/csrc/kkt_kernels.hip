// All-at-once matrix of eq. (FinalA), its right-hand side (section 2.2) and
// the FP64 vector kernels of the outer Krylov method.
//
// Canonical layout: x[b][t][v_x (2N+1)^2, v_y (2N+1)^2, p (N+1)^2].
// Rows (section 2.2, one backward-Euler step per block, t = 0..nt-1 here):
//   adjoint momentum  (b=0): tau M v_t + M (l_t - l_{t+1}) + tau L^T l_t + tau B^T mu_t
//   adjoint divergence(b=0): tau B l_t
//   state momentum    (b=1): M (v_t - v_{t-1}) + tau L v_t + tau B^T p_t - tau/beta M l_t
//   state divergence  (b=1): tau B v_t
// with v_{-1} = 0, l_{nt} = 0, L = nu K + N(w), the pinned pressure row and
// the Dirichlet velocity rows zero.
#include <type_traits>

#include "kernels.h"

namespace pintoc {

// Entry (k, j = 2k + off) of the 1-D mixed Q1-Q2 mass (m) and derivative (g)
// rows, the same values as mixed_rows(k) at index off + 2 (zero outside).
__device__ __forceinline__ void mixed_at(int k, int off, int n, double h, double& m, double& g) {
  m = 0.0;
  g = 0.0;
  if (k < 0 || k > n || off < -2 || off > 2) return;
  const bool lo = k > 0, hi = k < n;
  switch (off) {
    case -2: g = lo ? -1.0 / 6.0 : 0.0; break;
    case -1: m = lo ? h / 3.0 : 0.0; g = lo ? -2.0 / 3.0 : 0.0; break;
    case 0: m = (lo ? h / 6.0 : 0.0) + (hi ? h / 6.0 : 0.0); g = (lo ? 5.0 / 6.0 : 0.0) + (hi ? -5.0 / 6.0 : 0.0); break;
    case 1: m = hi ? h / 3.0 : 0.0; g = hi ? 2.0 / 3.0 : 0.0; break;
    default: g = hi ? 1.0 / 6.0 : 0.0; break;
  }
}

// Oseen: momentum and divergence rows of one block row b at one time step t
// on LDS tiles.  A work-group owns 64 x 32 interior Q2 nodes and the Q1 nodes whose
// mixed stencils (Q2 nodes 2k - 2 .. 2k + 2 per direction) fall inside its
// staged window: Q1 columns [32 bx + 1, 32 bx + 33) (from 0 in the first tile
// column, up to n in the last), rows likewise with 16.  Per velocity
// component it stages, over the tile and a two-node halo,
//   F = ca v_t + cb l_t - un   (the field the mass matrix acts on)
//   U = l_t (b = 0) or v_t (b = 1)   (the field K, N and B act on)
// with all 30 global loads of a thread issued before the first is used, and
// once per work-group the 35 x 19 Q1 window of the pressure field of B^T
// (mu_t for b = 0, p_t for b = 1).  Thread (column, strip of 8 rows) walks
// its strip keeping the x-sums (m' on F, k' and m' on U) of the five rows
// around the output row in registers; B^T reads the Q1 window; the Oseen
// convection stencil reads its 25 entries per node from an entry-major table
// (coalesced) and U.  The divergence rows accumulate both components' B
// terms over U in registers and are written after the second component.
// The Dirichlet ring of the velocity rows is written by k_kkt_ring.
constexpr int kVTX = 64, kVTY = 32, kVTS = 8;
constexpr int kVLX = kVTX + 4, kVLY = kVTY + 4, kVLN = kVLX * kVLY;
constexpr int kPLX = kVTX / 2 + 3, kPLY = kVTY / 2 + 3, kPLN = kPLX * kPLY;
constexpr int kVIt = (kVLN + 255) / 256, kPIt = (kPLN + 255) / 256;
constexpr int kDivPer = 3;                                   // owned Q1 nodes per thread (33 x 17 <= 3 x 256)
static_assert((kVTX / 2 + 1) * (kVTY / 2 + 1) <= kDivPer * 256, "divergence rows per thread");
static_assert(kVTY == 4 * kVTS, "four strips of rows per tile");

__global__ __launch_bounds__(256, 3) void k_kkt_tile(const double* __restrict__ x, double* __restrict__ y, int n, int nt,
                                                  double tau, double beta, double nu,
                                                  const double* __restrict__ convT, int ntx) {
  __shared__ double F[kVLN], U[kVLN], Q[kPLN], D[kDivPer * 256];
  const int nq = 2 * n + 1, nq2 = nq * nq, np = n + 1, np2 = np * np;
  const int L = 2 * nq2 + np2;
  const int b = blockIdx.y, t = blockIdx.z;
  const int bx = blockIdx.x % ntx, by = blockIdx.x / ntx;
  const int x0 = 1 + bx * kVTX, y0 = 1 + by * kVTY;          // first interior output node of the tile
  const int qx0 = (x0 >> 1) - 1, qy0 = (y0 >> 1) - 1;        // first staged Q1 node
  const double h = 1.0 / n;
  const double* X0 = x + (size_t)t * L;                      // v_t, p_t
  const double* X1 = x + (size_t)(nt + t) * L;               // l_t, mu_t
  const bool has_un = b == 0 ? t + 1 < nt : t > 0;
  const double* UN = b == 0 ? X1 + (has_un ? L : 0) : X0 - (has_un ? L : 0);   // l_{t+1} or v_{t-1}
  const double ca = b == 0 ? tau : 1.0, cb = b == 0 ? 1.0 : -tau / beta;
  // pressure field of B^T into Q (zero outside [0, n]^2)
  {
    const double* pf = (b == 0 ? X1 : X0) + 2 * nq2;
    double qv[kPIt];
#pragma unroll
    for (int k = 0; k < kPIt; ++k) {
      const int e = threadIdx.x + 256 * k, ly = e / kPLX, lx = e - ly * kPLX;
      const int gx = qx0 + lx, gy = qy0 + ly;
      const bool in = e < kPLN && gx >= 0 && gx <= n && gy >= 0 && gy <= n;
      const double v = pf[(size_t)min(max(gy, 0), n) * np + min(max(gx, 0), n)];
      qv[k] = in ? v : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kPIt; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < kPLN) Q[e] = qv[k];
    }
  }
  const int lx = threadIdx.x & (kVTX - 1), strip = threadIdx.x / kVTX;
  const int ix = x0 + lx;
  double mx[5], kx[5], my[5], ky[5];
  q2_rows(ix, h, mx, kx);
  const int kx0 = (ix >> 1) - 1;
  double wbm[3], wbg[3];                                     // mixed mass / derivative weights along x
#pragma unroll
  for (int c = 0; c < 3; ++c) mixed_at(kx0 + c, ix - 2 * (kx0 + c), n, h, wbm[c], wbg[c]);
  const int r0 = strip * kVTS;                               // first output row of the strip (tile-local)
  // owned Q1 nodes
  const int kxb = bx == 0 ? 0 : qx0 + 2, kxe = min(qx0 + 2 + kVTX / 2, n + 1);
  const int kyb = by == 0 ? 0 : qy0 + 2, kye = min(qy0 + 2 + kVTY / 2, n + 1);
  const int nkx = kxe - kxb, nk = nkx * (kye - kyb);
#pragma unroll
  for (int i = 0; i < kDivPer; ++i) D[threadIdx.x + 256 * i] = 0.0;   // divergence sums, one slot per owned node
  double* Y = y + ((size_t)b * nt + t) * L;
#pragma unroll 1
  for (int comp = 0; comp < 2; ++comp) {
    const double* vt = X0 + comp * nq2;
    const double* lt = X1 + comp * nq2;
    const double* un = UN + comp * nq2;
    double fv[kVIt], uv[kVIt];
#pragma unroll
    for (int k = 0; k < kVIt; ++k) {
      const int e = threadIdx.x + 256 * k, ly = e / kVLX, lxs = e - ly * kVLX;
      const int gx = x0 - 2 + lxs, gy = y0 - 2 + ly;
      const bool in = e < kVLN && gx >= 0 && gx < nq && gy >= 0 && gy < nq;
      const size_t o = (size_t)min(max(gy, 0), nq - 1) * nq + min(max(gx, 0), nq - 1);
      const double vv = vt[o], ll = lt[o], uu = un[o];
      fv[k] = in ? ca * vv + cb * ll - (has_un ? uu : 0.0) : 0.0;
      uv[k] = in ? (b == 0 ? ll : vv) : 0.0;
    }
    if (comp) __syncthreads();                               // the previous component's reads are done
#pragma unroll
    for (int k = 0; k < kVIt; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < kVLN) {
        F[e] = fv[k];
        U[e] = uv[k];
      }
    }
    __syncthreads();
    // momentum rows of this component
    if (ix <= nq - 2) {
      double SM[5], SK[5], SU[5];
      auto sums = [&](int lr, double& sm, double& sk, double& su) {   // lr: staged row (0 = y0 - 2)
        const double* fr = F + lr * kVLX + lx;
        const double* ur = U + lr * kVLX + lx;
        sm = 0;
        sk = 0;
        su = 0;
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) {
          sm += mx[dx] * fr[dx];
          sk += kx[dx] * ur[dx];
          su += mx[dx] * ur[dx];
        }
      };
#pragma unroll
      for (int d = 0; d < 4; ++d) sums(r0 + d, SM[d], SK[d], SU[d]);
      double* yo = Y + comp * nq2;
#pragma unroll 1
      for (int i = 0; i < kVTS; ++i) {
        const int iy = y0 + r0 + i;
        sums(r0 + i + 4, SM[4], SK[4], SU[4]);
        if (iy <= nq - 2) {
          q2_rows(iy, h, my, ky);
          double mm = 0, kk = 0;
#pragma unroll
          for (int d = 0; d < 5; ++d) {
            mm += my[d] * SM[d];
            kk += my[d] * SK[d] + ky[d] * SU[d];
          }
          const int ky0 = (iy >> 1) - 1;
          double bt = 0.0;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            double m, g;
            mixed_at(ky0 + a, iy - 2 * (ky0 + a), n, h, m, g);
            const double* row = Q + (ky0 + a - qy0) * kPLX + (kx0 - qx0);
            const double rs = comp == 0 ? wbg[0] * row[0] + wbg[1] * row[1] + wbg[2] * row[2]
                                        : wbm[0] * row[0] + wbm[1] * row[1] + wbm[2] * row[2];
            bt += (comp == 0 ? m : g) * rs;
          }
          // convection: entries of N (b = 1) or N^T (b = 0) at this node, entry-major
          const double* ct = convT + (size_t)(b == 0 ? 25 : 0) * nq2 + (size_t)iy * nq + ix;
          double cc = 0.0;
#pragma unroll
          for (int dy = 0; dy < 5; ++dy) {
            const double* ur = U + (r0 + i + dy) * kVLX + lx;
#pragma unroll
            for (int dx = 0; dx < 5; ++dx) cc += ct[(size_t)(dy * 5 + dx) * nq2] * ur[dx];
          }
          yo[(size_t)iy * nq + ix] = mm + tau * nu * kk + tau * cc - tau * bt;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          SM[d] = SM[d + 1];
          SK[d] = SK[d + 1];
          SU[d] = SU[d + 1];
        }
      }
    }
    // divergence rows: this component's B term on U
#pragma unroll 1
    for (int e = threadIdx.x; e < nk; e += 256) {
      const int kyy = kyb + e / nkx, kxx = kxb + e % nkx;
      double wx[5], wy[5], w2[5];
      if (comp == 0) {
        mixed_rows(kxx, n, h, w2, wx);             // derivative along x
        mixed_rows(kyy, n, h, wy, w2);             // mass along y
      } else {
        mixed_rows(kxx, n, h, wx, w2);             // mass along x
        mixed_rows(kyy, n, h, w2, wy);             // derivative along y
      }
      // staged indices of Q2 nodes 2k - 2 .. 2k + 2 (those outside the window
      // only ever meet zero weights: clamp them)
      const int sx = 2 * kxx - x0, sy = 2 * kyy - y0;
      double s = 0.0;
#pragma unroll
      for (int dy = 0; dy < 5; ++dy) {
        const double* ur = U + min(max(sy + dy, 0), kVLY - 1) * kVLX;
        double rs = 0.0;
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) rs += wx[dx] * ur[min(max(sx + dx, 0), kVLX - 1)];
        s += wy[dy] * rs;
      }
      D[e] += s;
    }
  }
#pragma unroll 1
  for (int e = threadIdx.x; e < nk; e += 256) {
    const int kyy = kyb + e / nkx, kxx = kxb + e % nkx, k = kyy * np + kxx;
    Y[2 * nq2 + k] = k == 0 ? 0.0 : -tau * D[e];              // the pinned pressure row is zero
  }
}

// Stokes: the same rows with time stepping.  A work-group owns one tile of
// 64 x 16 interior Q2 nodes (with its Q1 nodes, chosen as above) for a span
// of tc consecutive time steps and walks them in order, staging each field
// once (v_t and l_t per component, p_t and mu_t) instead of once per block
// row and again as the neighbouring step's field.  By linearity the mass
// terms split into M v_t, M l_t of the current step, so a thread keeps per
// output node and component
//   MVp = M v_{t-1}                                  (state row at t)
//   AP  = tau M v_{t-1} + M l_{t-1} + tau nu K l_{t-1} + tau B^T mu_{t-1}
//                                                    (adjoint row at t-1, less M l_t)
// in registers: the state row at t is written in step t, the adjoint row at
// t - 1 in step t once M l_t is known.  A span starts one step early (M v
// only) and ends one step late (M l only) unless it touches t = 0 or nt.
// Row and column parities fix the 1-D weights, so M and K use the integer
// weights m', k' with the scales applied once.  The global loads of the next
// (step, component) phase are issued before the current phase computes, so
// HBM latency overlaps the stencil work.
constexpr int kSTX = 64, kSTY = 16, kSTS = 4;                // tile (interior Q2 nodes) and rows per thread
constexpr int kSLX = kSTX + 4, kSLY = kSTY + 4, kSLN = kSLX * kSLY;
constexpr int kSPX = kSTX / 2 + 3, kSPY = kSTY / 2 + 3, kSPN = kSPX * kSPY;
constexpr int kSVIt = (kSLN + 255) / 256, kSPIt = (kSPN + 255) / 256;
constexpr int kSDiv = 2;                                     // owned Q1 nodes per thread (33 x 9 <= 2 x 256)
static_assert((kSTX / 2 + 1) * (kSTY / 2 + 1) <= kSDiv * 256, "divergence rows per thread");
static_assert(kSTY == 4 * kSTS, "four strips of rows per tile");

struct SpanStage {
  double v[kSVIt], l[kSVIt], p[kSPIt], m[kSPIt];
};

// Issue the loads of step s, component c (v and/or l, and the two pressure
// fields when wq) into registers; out-of-grid nodes read as zero.
__device__ __forceinline__ void span_load(SpanStage& st, const double* __restrict__ x, int nq, int n, int L, int nt,
                                          int s, int c, bool wv, bool wl, bool wq, int x0, int y0, int qx0, int qy0) {
  const int nq2 = nq * nq, np = n + 1;
  const double* vs = x + (size_t)s * L + c * nq2;
  const double* ls = x + (size_t)(nt + s) * L + c * nq2;
  int tid = threadIdx.x;                 // recomputed offsets, not held across the step loop
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int k = 0; k < kSVIt; ++k) {
    const int e = tid + 256 * k, ly = e / kSLX, lxs = e - ly * kSLX;
    const int gx = x0 - 2 + lxs, gy = y0 - 2 + ly;
    const bool in = e < kSLN && gx >= 0 && gx < nq && gy >= 0 && gy < nq;
    const size_t o = (size_t)min(max(gy, 0), nq - 1) * nq + min(max(gx, 0), nq - 1);
    if (wv) st.v[k] = in ? vs[o] : 0.0;
    if (wl) st.l[k] = in ? ls[o] : 0.0;
  }
  if (wq) {
    const double* ps = x + (size_t)s * L + 2 * nq2;
    const double* ms = x + (size_t)(nt + s) * L + 2 * nq2;
#pragma unroll
    for (int k = 0; k < kSPIt; ++k) {
      const int e = tid + 256 * k, ly = e / kSPX, lx = e - ly * kSPX;
      const int gx = qx0 + lx, gy = qy0 + ly;
      const bool in = e < kSPN && gx >= 0 && gx <= n && gy >= 0 && gy <= n;
      const size_t o = (size_t)min(max(gy, 0), n) * np + min(max(gx, 0), n);
      st.p[k] = in ? ps[o] : 0.0;
      st.m[k] = in ? ms[o] : 0.0;
    }
  }
}

__device__ __forceinline__ void span_store(const SpanStage& st, double* V, double* Lm, double* QP, double* QM, bool wv,
                                           bool wl, bool wq) {
#pragma unroll
  for (int k = 0; k < kSVIt; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < kSLN) {
      if (wv) V[e] = st.v[k];
      if (wl) Lm[e] = st.l[k];
    }
  }
  if (wq) {
#pragma unroll
    for (int k = 0; k < kSPIt; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < kSPN) {
        QP[e] = st.p[k];
        QM[e] = st.m[k];
      }
    }
  }
}

// Uniform scalars of k_kkt_span, computed on the host (kernel arguments stay
// in scalar registers instead of occupying vector registers).
struct SpanScal {
  double tau, tb, tn, h, smm, smk, h3, c16, c23;   // tau, tau/beta, tau nu, h, (h/30)^2, (h/30)/(3h), h/3, 1/6, 2/3
};

__global__ __launch_bounds__(256, 2) void k_kkt_span(const double* __restrict__ x, double* __restrict__ y, int n,
                                                     int nt, SpanScal sc, int ntx, int ntiles, int tc) {
  // DV, DL: divergence sums of the Q1 nodes on the grid's boundary (indexed
  // like the owned nodes); IV, IL: those of interior Q1 nodes, per thread and
  // vertex row of its strip
  __shared__ double V[kSLN], Lm[kSLN], QP[kSPN], QM[kSPN], DV[kSDiv * 256], DL[kSDiv * 256];
  __shared__ double IV[(kSTS / 2) * 256], IL[(kSTS / 2) * 256];
  const int nq = 2 * n + 1, nq2 = nq * nq, np = n + 1, np2 = np * np;
  const int L = 2 * nq2 + np2;
  // Work-group ids are dealt round-robin to the 8 XCDs; id g takes item
  // v = (g % 8) (G / 8) + g / 8, so each XCD holds a contiguous range of v,
  // i.e. a compact block of tiles (row-major, spans fastest): neighbouring
  // tiles of one span share their halo lines in that XCD's L2.
  const int nspan = (nt + tc - 1) / tc;
  const unsigned v = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if (v >= (unsigned)(ntiles * nspan)) return;                 // whole work-group: no barrier is skipped
  const int tile = (int)(v / nspan), span = (int)(v % nspan);
  const int bx = tile % ntx, by = tile / ntx;
  const int x0 = 1 + bx * kSTX, y0 = 1 + by * kSTY;
  const int qx0 = (x0 >> 1) - 1, qy0 = (y0 >> 1) - 1;
  const int t0 = span * tc, t1 = min(t0 + tc, nt);
  const int sb = t0 > 0 ? t0 - 1 : t0, se = t1 < nt ? t1 : t1 - 1;
  const double tau = sc.tau, tb = sc.tb, tn = sc.tn, h = sc.h;
  const bool ring = bx == 0 || bx == ntx - 1 || by == 0 || (by + 1) * kSTY >= 2 * n - 1;   // tile on the grid edge
#pragma unroll
  for (int i = 0; i < kSDiv; ++i) {
    DV[threadIdx.x + 256 * i] = 0.0;
    DL[threadIdx.x + 256 * i] = 0.0;
  }
  double MVp[2][kSTS], AP[2][kSTS];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < kSTS; ++i) {
      MVp[c][i] = 0.0;
      AP[c][i] = 0.0;
    }

  // one (step, component) phase over the staged fields
  auto phase = [&](int s, auto cc) {
    constexpr int c = decltype(cc)::value;
    const bool pro = s < t0, epi = s >= t1;
    // Per-lane geometry, recomputed in every phase from a thread index the
    // compiler may not treat as loop-invariant: hoisting these values (and the
    // addresses derived from them) out of the step loop would hold far more
    // registers than recomputing them costs.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lx = tid & (kSTX - 1);
    const int r0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kSTX) * kSTS;   // wave-uniform strip
    const int ix = x0 + lx;
    const bool colin = ix <= nq - 2;
    // integer x-weights of the column (vertex: m' = (-1, 2, 8, 2, -1), k' = (1, -8, 14, -8, 1);
    // midpoint: m' = (0, 2, 16, 2, 0), k' = (0, -8, 16, -8, 0)); the scales h/30 and
    // 1/(3h) are applied with the y-weights
    const bool xvert = (ix & 1) == 0;
    const double m04 = xvert ? -1.0 : 0.0, m2 = xvert ? 8.0 : 16.0, k04 = xvert ? 1.0 : 0.0, k2 = xvert ? 14.0 : 16.0;
    const int kx0 = (ix >> 1) - 1;
    if (colin) {
      // x-sums per staged row: m' v, k' v, m' l, k' l, and the mixed x-sums of
      // the divergence rows (derivative weights for c = 0, mass for c = 1) that
      // a Q1 node kx takes from the five Q2 nodes around 2 kx = ix (used by the
      // lanes of even ix)
      double S[5][6];
      auto sums = [&](int lr, double* o) {
        const double* vr = V + lr * kSLX + lx;
        const double* lr_ = Lm + lr * kSLX + lx;
        const double v04 = vr[0] + vr[4], v13 = vr[1] + vr[3], l04 = lr_[0] + lr_[4], l13 = lr_[1] + lr_[3];
        o[0] = fma(m04, v04, fma(2.0, v13, m2 * vr[2]));
        o[1] = fma(k04, v04, fma(-8.0, v13, k2 * vr[2]));
        o[2] = fma(m04, l04, fma(2.0, l13, m2 * lr_[2]));
        o[3] = fma(k04, l04, fma(-8.0, l13, k2 * lr_[2]));
        if (c == 0) {
          o[4] = fma(sc.c16, vr[4] - vr[0], sc.c23 * (vr[3] - vr[1]));
          o[5] = fma(sc.c16, lr_[4] - lr_[0], sc.c23 * (lr_[3] - lr_[1]));
        } else {
          o[4] = sc.h3 * (vr[1] + vr[2] + vr[3]);
          o[5] = sc.h3 * (lr_[1] + lr_[2] + lr_[3]);
        }
      };
#pragma unroll
      for (int d = 0; d < 4; ++d) sums(r0 + d, S[d]);
      double* Ys = y + ((size_t)(nt + s)) * L + c * nq2;       // state rows at s
      double* Ya = y + (size_t)max(s - 1, 0) * L + c * nq2;    // adjoint rows at s - 1 (s > 0 when written)
      double* Yl = y + (size_t)s * L + c * nq2;                // adjoint rows at s (s = nt - 1)
      // Output row iy = y0 + r0 + i has the parity of i + 1 (y0 odd, r0 even),
      // so its 1-D Q2 weights (h/30 m', 1/(3h) k') and, for an interior row,
      // its mixed weights over the Q1 rows around it are fixed per i.
      const double smm = sc.smm, smk = sc.smk, h3 = sc.h3;
#pragma unroll
      for (int i = 0; i < kSTS; ++i) {
        const int iy = y0 + r0 + i;
        sums(r0 + i + 4, S[4]);
        if (iy <= nq - 2) {
          const bool vert = (i & 1) == 1;            // iy even: a vertex row
          double MV, KV, ML, KL;
          {
            double a0, a1, a2, a3, b0, b2;           // m'-combinations of the four sums, k'-combinations of m-sums
            if (vert) {
              // integer weights by exponent shifts (exact) and inline constants
              a0 = ldexp(S[2][0], 3) + 2 * (S[1][0] + S[3][0]) - (S[0][0] + S[4][0]);
              a1 = ldexp(S[2][1], 3) + 2 * (S[1][1] + S[3][1]) - (S[0][1] + S[4][1]);
              a2 = ldexp(S[2][2], 3) + 2 * (S[1][2] + S[3][2]) - (S[0][2] + S[4][2]);
              a3 = ldexp(S[2][3], 3) + 2 * (S[1][3] + S[3][3]) - (S[0][3] + S[4][3]);
              b0 = fma(-2.0, S[2][0], ldexp(S[2][0], 4)) - ldexp(S[1][0] + S[3][0], 3) + (S[0][0] + S[4][0]);
              b2 = fma(-2.0, S[2][2], ldexp(S[2][2], 4)) - ldexp(S[1][2] + S[3][2], 3) + (S[0][2] + S[4][2]);
            } else {
              a0 = ldexp(S[2][0], 4) + 2 * (S[1][0] + S[3][0]);
              a1 = ldexp(S[2][1], 4) + 2 * (S[1][1] + S[3][1]);
              a2 = ldexp(S[2][2], 4) + 2 * (S[1][2] + S[3][2]);
              a3 = ldexp(S[2][3], 4) + 2 * (S[1][3] + S[3][3]);
              b0 = ldexp(S[2][0], 4) - ldexp(S[1][0] + S[3][0], 3);
              b2 = ldexp(S[2][2], 4) - ldexp(S[1][2] + S[3][2], 3);
            }
            MV = smm * a0;
            KV = smk * (a1 + b0);
            ML = smm * a2;
            KL = smk * (a3 + b2);
          }
          const size_t o = (size_t)iy * nq + ix;
          if (pro) {
            MVp[c][i] = MV;
          } else if (epi) {
            Ya[o] = AP[c][i] - ML;
          } else {
            // B^T: Q1 rows around iy with their mixed mass (m) / derivative (g) weights
            const int kr = (iy >> 1) - 1 - qy0;          // window row of Q1 row (iy >> 1) - 1
            const int qo = kr * kSPX + (kx0 - qx0);
            // x-weights of B^T over Q1 columns kx0 .. kx0 + 2 (derivative for c = 0,
            // mass for c = 1), fixed by the parity of the interior column ix
            double w[3];
            if (c == 0) {
              w[0] = xvert ? sc.c16 : 0.0;
              w[1] = xvert ? 0.0 : sc.c23;
              w[2] = xvert ? -sc.c16 : -sc.c23;
            } else {
              w[0] = 0.0;
              w[1] = sc.h3;
              w[2] = xvert ? 0.0 : sc.h3;
            }
            auto rowp = [&](const double* Q, int r) {
              return w[0] * Q[qo + r * kSPX] + w[1] * Q[qo + r * kSPX + 1] + w[2] * Q[qo + r * kSPX + 2];
            };
            double btp, btm;
            if (vert) {                                  // rows k-1, k, k+1: m = (0, h/3, 0), g = (1/6, 0, -1/6)
              if (c == 0) {
                btp = h3 * rowp(QP, 1);
                btm = h3 * rowp(QM, 1);
              } else {
                btp = sc.c16 * (rowp(QP, 0) - rowp(QP, 2));
                btm = sc.c16 * (rowp(QM, 0) - rowp(QM, 2));
              }
            } else {                                     // rows k, k+1: m = (h/3, h/3), g = (2/3, -2/3)
              if (c == 0) {
                btp = h3 * (rowp(QP, 1) + rowp(QP, 2));
                btm = h3 * (rowp(QM, 1) + rowp(QM, 2));
              } else {
                btp = sc.c23 * (rowp(QP, 1) - rowp(QP, 2));
                btm = sc.c23 * (rowp(QM, 1) - rowp(QM, 2));
              }
            }
            Ys[o] = MV - MVp[c][i] - tb * ML + tn * KV - tau * btp;
            MVp[c][i] = MV;
            const double ap = tau * MV + ML + tn * KL - tau * btm;
            if (s > t0) Ya[o] = AP[c][i] - ML;
            if (s == nt - 1) Yl[o] = ap;
            AP[c][i] = ap;
            if (vert) {
              // divergence rows of the interior Q1 node (ix / 2, iy / 2): the y-weights
              // of the rows iy - 2 .. iy + 2 are mass for c = 0 and derivative for c = 1
              const int slot = (i >> 1) * 256 + tid;
              if (c == 0) {
                IV[slot] = h3 * (S[1][4] + S[2][4] + S[3][4]);
                IL[slot] = h3 * (S[1][5] + S[2][5] + S[3][5]);
              } else if (xvert) {
                const double dv = IV[slot] + fma(sc.c16, S[4][4] - S[0][4], sc.c23 * (S[3][4] - S[1][4]));
                const double dl = IL[slot] + fma(sc.c16, S[4][5] - S[0][5], sc.c23 * (S[3][5] - S[1][5]));
                const size_t k = (size_t)(iy >> 1) * np + (ix >> 1);
                y[(size_t)(nt + s) * L + 2 * nq2 + k] = -tau * dv;       // state divergence
                y[(size_t)s * L + 2 * nq2 + k] = -tau * dl;              // adjoint divergence
              }
            }
          }
        }
#pragma unroll
        for (int d = 0; d < 4; ++d)
#pragma unroll
          for (int q = 0; q < 6; ++q) S[d][q] = S[d + 1][q];
      }
    }
    if (pro || epi || !ring) return;
    // divergence rows of the Q1 nodes on the grid's boundary (their Q2 centre
    // is no momentum output): this component's B terms on v_s and l_s
    const int kxb = bx == 0 ? 0 : qx0 + 2, kxe = min(qx0 + 2 + kSTX / 2, n + 1);
    const int kyb = by == 0 ? 0 : qy0 + 2, kye = min(qy0 + 2 + kSTY / 2, n + 1);
    const int nkx = kxe - kxb, nk = nkx * (kye - kyb);
#pragma unroll 1
    for (int e = tid; e < nk; e += 256) {
      const int kyy = kyb + e / nkx, kxx = kxb + e % nkx;
      if (kxx > 0 && kxx < n && kyy > 0 && kyy < n) continue;
      double wx[5], wy[5], w2[5];
      if (c == 0) {
        mixed_rows(kxx, n, h, w2, wx);
        mixed_rows(kyy, n, h, wy, w2);
      } else {
        mixed_rows(kxx, n, h, wx, w2);
        mixed_rows(kyy, n, h, w2, wy);
      }
      const int sx = 2 * kxx - x0, sy = 2 * kyy - y0;
      double sv = 0.0, sl = 0.0;
#pragma unroll
      for (int dy = 0; dy < 5; ++dy) {
        const int ro = min(max(sy + dy, 0), kSLY - 1) * kSLX;
        double rv = 0.0, rl = 0.0;
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) {
          const int q = ro + min(max(sx + dx, 0), kSLX - 1);
          rv += wx[dx] * V[q];
          rl += wx[dx] * Lm[q];
        }
        sv += wy[dy] * rv;
        sl += wy[dy] * rl;
      }
      if (c == 0) {
        DV[e] += sv;
        DL[e] += sl;
      } else {
        const int k = kyy * np + kxx;
        const double dv = DV[e] + sv, dl = DL[e] + sl;
        y[(size_t)(nt + s) * L + 2 * nq2 + k] = k == 0 ? 0.0 : -tau * dv;     // state divergence
        y[(size_t)s * L + 2 * nq2 + k] = k == 0 ? 0.0 : -tau * dl;            // adjoint divergence
        DV[e] = 0.0;
        DL[e] = 0.0;
      }
    }
  };

  SpanStage st;
  span_load(st, x, nq, n, L, nt, sb, 0, true, sb >= t0, sb >= t0, x0, y0, qx0, qy0);
#pragma unroll 1
  for (int s = sb; s <= se; ++s) {
    const bool pro = s < t0, epi = s >= t1, wq = !pro && !epi;
    const bool wv = !epi, wl = !pro;
    span_store(st, V, Lm, QP, QM, wv, wl, wq);
    __syncthreads();
    span_load(st, x, nq, n, L, nt, s, 1, wv, wl, false, x0, y0, qx0, qy0);
    phase(s, std::integral_constant<int, 0>{});
    __syncthreads();
    span_store(st, V, Lm, QP, QM, wv, wl, false);
    __syncthreads();
    if (s < se) {
      const bool npro = s + 1 < t0, nepi = s + 1 >= t1;
      span_load(st, x, nq, n, L, nt, s + 1, 0, !nepi, !npro, !npro && !nepi, x0, y0, qx0, qy0);
    }
    phase(s, std::integral_constant<int, 1>{});
    __syncthreads();
  }
}

// zero velocity rows on the Dirichlet ring of every grid (b, t, comp)
__global__ __launch_bounds__(256) void k_kkt_ring(double* __restrict__ y, int n, int nt) {
  const int nq = 2 * n + 1, nq2 = nq * nq, L = 2 * nq2 + (n + 1) * (n + 1);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 4 * (nq - 1)) return;
  const int t = blockIdx.y, bc = blockIdx.z, b = bc >> 1, comp = bc & 1;
  const int side = e / (nq - 1), k = e - side * (nq - 1);
  int ix, iy;
  switch (side) {
    case 0: ix = k; iy = 0; break;
    case 1: ix = nq - 1; iy = k; break;
    case 2: ix = nq - 1 - k; iy = nq - 1; break;
    default: ix = 0; iy = nq - 1 - k; break;
  }
  y[((size_t)b * nt + t) * L + comp * nq2 + (size_t)iy * nq + ix] = 0.0;
}

// b = tau M v_d on the adjoint momentum rows, zero elsewhere.
__global__ __launch_bounds__(256) void k_assemble_rhs(const double* __restrict__ vd, double* __restrict__ out, int n, int nt, double tau) {
  const int nq = 2 * n + 1, nq2 = nq * nq, np = n + 1, np2 = np * np;
  const int L = 2 * nq2 + np2;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y, b = blockIdx.z;
  if (g >= L) return;
  double v = 0;
  if (b == 0 && g < 2 * nq2) {
    const int comp = g >= nq2, node = g - comp * nq2;
    const int ix = node % nq, iy = node / nq;
    if (ix > 0 && iy > 0 && ix < nq - 1 && iy < nq - 1) {
      double mx[5], kx[5], my[5], ky[5];
      const double h = 1.0 / n;
      q2_rows(ix, h, mx, kx);
      q2_rows(iy, h, my, ky);
      // boundary values of v_d are ignored: read them as zero
      double s = 0;
      const double* u = vd + ((size_t)t * 2 + comp) * nq2;
      for (int dy = 0; dy < 5; ++dy) {
        const int jy = iy + dy - 2;
        if (jy <= 0 || jy >= nq - 1) continue;
        double sm = 0;
        for (int dx = 0; dx < 5; ++dx) {
          const int jx = ix + dx - 2;
          if (jx <= 0 || jx >= nq - 1) continue;
          sm += mx[dx] * u[jy * nq + jx];
        }
        s += my[dy] * sm;
      }
      v = tau * s;
    }
  }
  out[((size_t)b * nt + t) * L + g] = v;
}

// Right-hand side for general data (section 2.2: the vectors g and h that
// collect forcing, boundary and initial values).  With the velocity at t_k
// split into the unknown interior part and the known boundary values h_k^B,
// the known terms of the discrete equations move to the right:
//   adjoint momentum (b=0): tau M (v_d,k - h_k^B)
//   adjoint divergence     : 0
//   state momentum   (b=1): tau M f_k - (M + tau L) h_k^B + M w_{k-1},
//                           w_0 = v_0 (interior) + h_0^B, w_{k-1} = h_{k-1}^B
//   state divergence       : -tau B h_k^B
// evaluated with the full-grid matrices (boundary columns included) on the
// interior rows.  Inputs are full Q2 nodal grids (NULL = zero): vd, f
// [nt][2][nq2] at t_1..t_nt, hb [nt+1][2][nq2] at t_0..t_nt (boundary entries
// read), v0 [2][nq2] (interior entries read).  Level t of the output is t_{t+1}.
__global__ __launch_bounds__(256) void k_rhs_data(const double* __restrict__ vd, const double* __restrict__ f,
                                                  const double* __restrict__ hb, const double* __restrict__ v0,
                                                  double* __restrict__ out, int n, int nt, double tau, double nu,
                                                  const double* __restrict__ conv) {
  const int nq = 2 * n + 1, nq2 = nq * nq, np = n + 1, np2 = np * np;
  const int L = 2 * nq2 + np2;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y, b = blockIdx.z;
  if (g >= L) return;
  const double h = 1.0 / n;
  auto on_bd = [&](int jx, int jy) { return jx == 0 || jy == 0 || jx == nq - 1 || jy == nq - 1; };
  // boundary value of the Dirichlet data at time level k (0..nt), component c
  auto hval = [&](int k, int c, int jx, int jy) {
    return (hb && on_bd(jx, jy)) ? hb[((size_t)k * 2 + c) * nq2 + (size_t)jy * nq + jx] : 0.0;
  };
  auto grid = [&](const double* a, int k, int c, int jx, int jy) {
    return a ? a[((size_t)k * 2 + c) * nq2 + (size_t)jy * nq + jx] : 0.0;
  };
  double v = 0;
  if (g < 2 * nq2) {
    const int comp = g >= nq2, node = g - comp * nq2;
    const int ix = node % nq, iy = node / nq;
    if (!on_bd(ix, iy)) {
      double mx[5], kx[5], my[5], ky[5];
      q2_rows(ix, h, mx, kx);
      q2_rows(iy, h, my, ky);
      const double* cn = (conv && b == 1) ? conv + (size_t)node * 50 : nullptr;     // N (not N^T)
      double mm = 0, kk = 0, cc = 0;
      for (int dy = 0; dy < 5; ++dy) {
        const int jy = iy + dy - 2;
        if (jy < 0 || jy >= nq) continue;
        double sm = 0, sk = 0, su = 0;
        for (int dx = 0; dx < 5; ++dx) {
          const int jx = ix + dx - 2;
          if (jx < 0 || jx >= nq) continue;
          const double hk = hval(t + 1, comp, jx, jy);
          double fm;
          if (b == 0) {
            fm = grid(vd, t, comp, jx, jy) - hk;
          } else {
            double wp;
            if (t == 0) wp = on_bd(jx, jy) ? hval(0, comp, jx, jy) : (v0 ? v0[(size_t)comp * nq2 + (size_t)jy * nq + jx] : 0.0);
            else wp = hval(t, comp, jx, jy);
            fm = tau * grid(f, t, comp, jx, jy) - hk + wp;
          }
          sm += mx[dx] * fm;
          sk += kx[dx] * hk;
          su += mx[dx] * hk;
          if (cn) cc += cn[dy * 5 + dx] * hk;
        }
        mm += my[dy] * sm;
        kk += my[dy] * sk + ky[dy] * su;
      }
      v = b == 0 ? tau * mm : mm - tau * (nu * kk + cc);
    }
  } else if (b == 1) {
    const int k = g - 2 * nq2, kx = k % np, ky = k / np;
    if (k != 0 && hb) {
      // -tau (B h^B)_k, B = negative divergence: B v = -(int psi_k d/dx v_x + int psi_k d/dy v_y)
      double mxx[5], gxx[5], mxy[5], gxy[5];
      mixed_rows(kx, n, h, mxx, gxx);
      mixed_rows(ky, n, h, mxy, gxy);
      double sdiv = 0;
      for (int dy = 0; dy < 5; ++dy) {
        const int jy = 2 * ky + dy - 2;
        if (jy < 0 || jy >= nq) continue;
        for (int dx = 0; dx < 5; ++dx) {
          const int jx = 2 * kx + dx - 2;
          if (jx < 0 || jx >= nq) continue;
          sdiv += mxy[dy] * gxx[dx] * hval(t + 1, 0, jx, jy) + gxy[dy] * mxx[dx] * hval(t + 1, 1, jx, jy);
        }
      }
      v = tau * sdiv;                       // -tau * (-sdiv)
    }
  }
  out[((size_t)b * nt + t) * L + g] = v;
}

// y = diag(sv on velocity entries, sp on pressure entries) x over both blocks
// and every time level; y may equal x.
__global__ __launch_bounds__(256) void k_scale_canon(double* y, const double* x, int n, int nt, double sv, double sp) {
  const int nq = 2 * n + 1, nq2 = nq * nq, L = 2 * nq2 + (n + 1) * (n + 1);
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= L) return;
  const size_t i = (size_t)blockIdx.y * L + g;
  y[i] = x[i] * (g < 2 * nq2 ? sv : sp);
}

void launch_rhs_data(hipStream_t s, const double* vd, const double* f, const double* hb, const double* v0, double* b,
                     int n, int nt, double tau, double nu, const double* conv) {
  const int L = 2 * (2 * n + 1) * (2 * n + 1) + (n + 1) * (n + 1);
  hipLaunchKernelGGL(k_rhs_data, dim3((L + 255) / 256, nt, 2), dim3(256), 0, s, vd, f, hb, v0, b, n, nt, tau, nu, conv);
}

void launch_scale_canon(hipStream_t s, double* y, const double* x, int n, int nt, double sv, double sp) {
  const int L = 2 * (2 * n + 1) * (2 * n + 1) + (n + 1) * (n + 1);
  hipLaunchKernelGGL(k_scale_canon, dim3((L + 255) / 256, 2 * nt), dim3(256), 0, s, y, x, n, nt, sv, sp);
}

// Time steps per span of k_kkt_span: long spans save the extra first and
// last step of each span, short ones give more work-groups; aim at about 512
// work-groups (two resident per CU), spans of 4 to 32 steps.  (At N = 128,
// nt = 256 spans of 8, 16 and 32 steps took 0.53, 0.52 and 0.50 ms.)
static int kkt_span_steps(int tiles, int nt) {
  int tc = 4;
  while (tc < 32 && (long)tiles * ((nt + 2 * tc - 1) / (2 * tc)) >= 512) tc *= 2;
  return tc;
}

void launch_kkt_apply(hipStream_t s, const double* x, double* y, int n, int nt, double tau, double beta, double nu,
                      const double* convT) {
  const int nq = 2 * n + 1, L = 2 * nq * nq + (n + 1) * (n + 1);
  (void)L;
  // momentum and divergence rows on LDS tiles, then the Dirichlet ring of the
  // momentum rows
  if (convT) {                // Oseen: one work-group per (tile, block row, step)
    const int ntx = (nq - 2 + kVTX - 1) / kVTX, nty = (nq - 2 + kVTY - 1) / kVTY;
    hipLaunchKernelGGL(k_kkt_tile, dim3(ntx * nty, 2, nt), dim3(256), 0, s, x, y, n, nt, tau, beta, nu, convT, ntx);
  } else {                    // Stokes: one work-group per (tile, span of tc steps)
    const int ntx = (nq - 2 + kSTX - 1) / kSTX, nty = (nq - 2 + kSTY - 1) / kSTY;
    const int tc = kkt_span_steps(ntx * nty, nt);
    const double h = 1.0 / n;
    const SpanScal sc{tau, tau / beta, tau * nu, h, (h / 30.0) * (h / 30.0), (h / 30.0) / (3.0 * h), h / 3.0,
                      1.0 / 6.0, 2.0 / 3.0};
    const int items = ntx * nty * ((nt + tc - 1) / tc);
    hipLaunchKernelGGL(k_kkt_span, dim3((items + 7) / 8 * 8), dim3(256), 0, s, x, y, n, nt, sc, ntx, ntx * nty, tc);
  }
  hipLaunchKernelGGL(k_kkt_ring, dim3((4 * (nq - 1) + 255) / 256, nt, 4), dim3(256), 0, s, y, n, nt);
}

void launch_assemble_rhs(hipStream_t s, const double* vd, double* b, int n, int nt, double tau) {
  const int L = 2 * (2 * n + 1) * (2 * n + 1) + (n + 1) * (n + 1);
  hipLaunchKernelGGL(k_assemble_rhs, dim3((L + 255) / 256, nt, 2), dim3(256), 0, s, vd, b, n, nt, tau);
}

// ---------------------------------------------------------------- BLAS
// Multi-dot: out[i] = <V_i, w>, i < k, V_i = V + i*ld.  Deterministic: every
// block reduces its slice in a fixed tree order into part[i][block]; a second
// kernel sums each row of part sequentially.
constexpr int kDotBlocks = 1024;
constexpr int kMaxDots = 40;

template <int K>
__global__ __launch_bounds__(256) void k_mdot(const double* __restrict__ V, size_t ld, int k, const double* __restrict__ w, size_t n,
                       double* __restrict__ part) {
  __shared__ double red[256];
  double acc[K];
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = 0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const double we = w[e];
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (i < k) acc[i] += V[i * ld + e] * we;
  }
  for (int i = 0; i < k && i < K; ++i) {
    red[threadIdx.x] = acc[i];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)i * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_rowsum(const double* __restrict__ part, int nblk, int k, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)i * nblk + b];
  out[i] = s;
}

// w -= sum_i c[i] V_i   (c on device)
__global__ __launch_bounds__(256) void k_mgs_update(double* __restrict__ w, const double* __restrict__ V, size_t ld, int k,
                             const double* __restrict__ c, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double s = w[e];
    for (int i = 0; i < k; ++i) s -= c[i] * V[i * ld + e];
    w[e] = s;
  }
}

// y = a x + b y
__global__ __launch_bounds__(256) void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a, double b, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + b * y[e];
}

// y += sum_i c[i] Z_i  (c on device)
__global__ __launch_bounds__(256) void k_lincomb_add(double* __restrict__ y, const double* __restrict__ Z, size_t ld, int k,
                              const double* __restrict__ c, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double s = y[e];
    for (int i = 0; i < k; ++i) s += c[i] * Z[i * ld + e];
    y[e] = s;
  }
}

void launch_mdot(hipStream_t s, const double* V, size_t ld, int k, const double* w, size_t n, double* part,
                 double* out) {
  for (int i0 = 0; i0 < k; i0 += 8) {
    const int kk = k - i0 < 8 ? k - i0 : 8;
    hipLaunchKernelGGL(k_mdot<8>, dim3(kDotBlocks), dim3(256), 0, s, V + i0 * ld, ld, kk, w, n, part);
    hipLaunchKernelGGL(k_rowsum, dim3(1), dim3(64), 0, s, part, kDotBlocks, kk, out + i0);
  }
}

void launch_mgs_update(hipStream_t s, double* w, const double* V, size_t ld, int k, const double* c, size_t n) {
  hipLaunchKernelGGL(k_mgs_update, dim3(2048), dim3(256), 0, s, w, V, ld, k, c, n);
}

void launch_axpby(hipStream_t s, double* y, const double* x, double a, double b, size_t n) {
  hipLaunchKernelGGL(k_axpby, dim3(2048), dim3(256), 0, s, y, x, a, b, n);
}

// y = a x + b z + c y (the three-term updates of MINRES)
__global__ __launch_bounds__(256) void k_axpbypcz(double* __restrict__ y, const double* __restrict__ x,
                                                  const double* __restrict__ z, double a, double b, double c,
                                                  size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * z[i] + c * y[i];
}

void launch_axpbypcz(hipStream_t s, double* y, const double* x, const double* z, double a, double b, double c,
                     size_t n) {
  hipLaunchKernelGGL(k_axpbypcz, dim3(2048), dim3(256), 0, s, y, x, z, a, b, c, n);
}

void launch_lincomb_add(hipStream_t s, double* y, const double* Z, size_t ld, int k, const double* c, size_t n) {
  hipLaunchKernelGGL(k_lincomb_add, dim3(2048), dim3(256), 0, s, y, Z, ld, k, c, n);
}

// FP32 copy of a vector (the FP32 outer basis: z is stored after its matvec)
__global__ __launch_bounds__(256) void k_to_f32(float* __restrict__ y, const double* __restrict__ x, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = (float)x[e];
}

// y += sum_i c[i] Z_i with FP32 Z, accumulated in FP64 (c on device)
__global__ __launch_bounds__(256) void k_lincomb_add_f32(double* __restrict__ y, const float* __restrict__ Z,
                                                         size_t ld, int k, const double* __restrict__ c, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double s = y[e];
    for (int i = 0; i < k; ++i) s += c[i] * (double)Z[i * ld + e];
    y[e] = s;
  }
}

void launch_to_f32(hipStream_t s, float* y, const double* x, size_t n) {
  hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(256), 0, s, y, x, n);
}

void launch_lincomb_add_f32(hipStream_t s, double* y, const float* Z, size_t ld, int k, const double* c, size_t n) {
  hipLaunchKernelGGL(k_lincomb_add_f32, dim3(2048), dim3(256), 0, s, y, Z, ld, k, c, n);
}

// zero-fill (a kernel rather than hipMemsetAsync so the sequence stays capturable)
__global__ __launch_bounds__(256) void k_fill_zero(uint4* __restrict__ p, size_t n16) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n16; e += (size_t)gridDim.x * blockDim.x)
    p[e] = make_uint4(0, 0, 0, 0);
}

void launch_fill_zero(hipStream_t s, void* p, size_t bytes) {
  // every buffer the library zeroes is carved 256-byte aligned and padded to a
  // multiple of 256 bytes, so rounding the length up to 16 bytes stays inside it
  hipLaunchKernelGGL(k_fill_zero, dim3(2048), dim3(256), 0, s, (uint4*)p, (bytes + 15) / 16);
}

}  // namespace pintoc
