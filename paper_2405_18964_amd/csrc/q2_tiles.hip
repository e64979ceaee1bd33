// Q2 tile kernels: the multicolour Gauss-Seidel sweep of the multigrid
// smoother (section 3.4) and the operator application / residual of
//   A = alpha M + gamma K + eta C      (C: one convection stencil table)
// on batches of padded Q2 grids (section 2.2), one 48 x 48 tile of one grid
// per work-group.
//
// LDS layout.  The tile and a halo of two nodes (52 x 52) are held as four
// parity sub-grids of 26 x 26 (x parity, y parity).  All nodes of one parity
// class have the same stencil shape (a vertex couples 5 nodes per direction,
// an edge midpoint 3) and the same integer 1-D weights
//   vertex    m = h/30 (-1, 2, 8, 2, -1),   k = 1/(3h) (1, -8, 14, -8, 1)
//   midpoint  m = h/30 (2, 16, 2),          k = 1/(3h) (-8, 16, -8)
// so M = h^2/900 (m' x m') and K = 1/90 (k' x m' + m' x k') in integer weights
// m', k' that the compiler folds into the code.  Each wave serves one class:
// wave (PX, PY) takes the nodes with gx % 2 == PX, gy % 2 == PY of the current
// colour, 8 x 8 of them per tile (one per 6 x 6 block); inside a sub-grid they
// sit 3 entries apart, so the 64 lanes' LDS reads fall on distinct banks.
//
// Colours and tiles are those of the tiled SOR: colour 3 (gy % 3) + gx % 3,
// tiles of 48 node indices aligned at node 0, Gauss-Seidel inside a tile and
// the values of the sweep's start for couplings to other tiles.
//
// Convection tables are reordered on the host per (tile, colour, class,
// stencil entry, lane), so the lanes of a wave read 64 consecutive doubles.
//
// Work-group order is XCD-aware: ids are dealt round-robin to the 8 XCDs, so
// id g is remapped to v = (g % 8) (G / 8) + g / 8 and every XCD gets a
// contiguous range of v.  With a convection table v runs over grids fastest
// (a tile's table stays in one XCD's L2 while every grid of the batch uses it);
// without one it runs over tiles fastest (neighbouring tiles share halo lines).
#include "kernels.h"

namespace pintoc {

namespace {

constexpr int kT = 48;            // tile side (node indices)
constexpr int kE = kT + 4;        // tile with halo
constexpr int kH = kE / 2;        // parity sub-grid side
constexpr int kSub = kH * kH;     // entries per sub-grid

__host__ __device__ constexpr int wlen(int P) { return P ? 3 : 5; }
__host__ __device__ constexpr int wlo(int P) { return P ? -1 : -2; }
__host__ __device__ constexpr int cm0(int P) { return P ? 16 : 8; }    // centre of m'
__host__ __device__ constexpr int ck0(int P) { return P ? 16 : 14; }   // centre of k'
// offset of a class's entries in the per-(tile, colour) convection block
__host__ __device__ constexpr int coff(int PX, int PY) { return PY ? (PX ? 55 : 40) : (PX ? 25 : 0); }

// LDS offset of neighbour (dx, dy) from the base of a class-(PX, PY) node
template <int PX, int PY>
__device__ __forceinline__ constexpr int loff(int dx, int dy) {
  return (((PY + dy) & 1) * 2 + ((PX + dx) & 1)) * kSub + ((PY + 2 + dy) >> 1) * kH + ((PX + 2 + dx) >> 1);
}

// (m' . v, k' . v) along one direction for class P
template <int P> struct Comb;
template <> struct Comb<0> {
  static __device__ __forceinline__ void run(const double* v, double& m, double& k) {
    const double s04 = v[0] + v[4], s13 = v[1] + v[3];
    m = fma(8.0, v[2], fma(2.0, s13, -s04));
    k = fma(14.0, v[2], fma(-8.0, s13, s04));
  }
};
template <> struct Comb<1> {
  static __device__ __forceinline__ void run(const double* v, double& m, double& k) {
    const double s02 = v[0] + v[2];
    m = fma(16.0, v[1], 2.0 * s02);
    k = fma(16.0, v[1], -8.0 * s02);
  }
};

// Tile-local coordinates of a lane's node of colour col in class (PX, PY).
template <int PX, int PY>
__device__ __forceinline__ void node_of(int col, int la, int lb, int& lx, int& ly) {
  const int cx = col % 3, cy = col / 3;
  lx = cx + 3 * (2 * la + ((PX - cx) & 1));
  ly = cy + 3 * (2 * lb + ((PY - cy) & 1));
}

// Uniform coefficients of a work-group: a = alpha h^2/900, g = gamma/90, e = eta.
struct TCoef {
  double ar, ai, gr, gi, er, ei;
};

__device__ __forceinline__ TCoef tcoef(const OpCoef& c, double h) {
  const double s = h * h / 900.0;
  return TCoef{c.alpha.x * s, c.alpha.y * s, c.gamma.x / 90.0, c.gamma.y / 90.0, c.eta.x, c.eta.y};
}

// a Md + g Kd: diagonal without convection for class (PX, PY)
template <int PX, int PY>
__device__ __forceinline__ double2 diag0(const TCoef& t) {
  constexpr double md = cm0(PX) * cm0(PY), kd = ck0(PX) * cm0(PY) + cm0(PX) * ck0(PY);
  return make_double2(t.ar * md + t.gr * kd, t.ai * md + t.gi * kd);
}

// A x at a class-(PX, PY) node: base points at the node's sub-grid origin, cn
// at its lane's first convection entry (stride 64).  Returns A x and the
// diagonal convection entry.
template <int PX, int PY, bool CV, typename R>
__device__ __forceinline__ double2 stencil(const cpx<R>* base, const double* __restrict__ cn, const TCoef& t,
                                          double& cdiag) {
  constexpr int nx = wlen(PX), ny = wlen(PY), lx0 = wlo(PX), ly0 = wlo(PY);
  double smr[ny], smi[ny], skr[ny], ski[ny];
  double cr = 0, ci = 0;
#pragma unroll
  for (int iy = 0; iy < ny; ++iy) {
    double vr[nx], vi[nx];
#pragma unroll
    for (int ix = 0; ix < nx; ++ix) {
      const cpx<R> v = base[loff<PX, PY>(lx0 + ix, ly0 + iy)];
      vr[ix] = (double)v.x;
      vi[ix] = (double)v.y;
      if (CV) {
        const double c = cn[(iy * nx + ix) * 64];
        cr = fma(c, vr[ix], cr);
        ci = fma(c, vi[ix], ci);
      }
    }
    Comb<PX>::run(vr, smr[iy], skr[iy]);
    Comb<PX>::run(vi, smi[iy], ski[iy]);
  }
  double pmr, pmi, kmr, kmi, mkr, mki, unr, uni;
  Comb<PY>::run(smr, pmr, kmr);        // m'_y . (m'_x v),  k'_y . (m'_x v)
  Comb<PY>::run(smi, pmi, kmi);
  Comb<PY>::run(skr, mkr, unr);        // m'_y . (k'_x v)
  Comb<PY>::run(ski, mki, uni);
  const double pkr = mkr + kmr, pki = mki + kmi;
  double axr = t.ar * pmr - t.ai * pmi + t.gr * pkr - t.gi * pki;
  double axi = t.ar * pmi + t.ai * pmr + t.gr * pki + t.gi * pkr;
  if (CV) {
    axr += t.er * cr - t.ei * ci;
    axi += t.er * ci + t.ei * cr;
    cdiag = cn[((wlen(PY) / 2) * nx + nx / 2) * 64];
  }
  return make_double2(axr, axi);
}

__device__ __forceinline__ bool tile_of_block(int ntiles, int nb, bool grid_fast, int& tile, int& f) {
  const unsigned per = gridDim.x >> 3;
  const unsigned v = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  if (v >= (unsigned)ntiles * (unsigned)nb) return false;
  if (grid_fast) { tile = (int)(v / nb); f = (int)(v % nb); }
  else { f = (int)(v / ntiles); tile = (int)(v % ntiles); }
  return true;
}

// (P e)(i, j) of the Q2 prolongation from the coarse padded grid (side nqc).
template <typename R>
__device__ __forceinline__ double2 q2_prolong_at(const cpx<R>* __restrict__ ec, int nqc, int i, int j) {
  auto w1 = [](int i, int& c0, double w[3]) {
    const int e = i >> 2, r = i & 3;
    c0 = 2 * e;
    if (r == 0) { w[0] = 1; w[1] = 0; w[2] = 0; }
    else if (r == 2) { w[0] = 0; w[1] = 1; w[2] = 0; }
    else if (r == 1) { w[0] = 0.375; w[1] = 0.75; w[2] = -0.125; }
    else { w[0] = -0.125; w[1] = 0.75; w[2] = 0.375; }
  };
  int cx0, cy0;
  double wx[3], wy[3];
  w1(i, cx0, wx);
  w1(j, cy0, wy);
  double sr = 0, si = 0;
  for (int a = 0; a < 3; ++a) {
    if (wy[a] == 0.0) continue;
    double rr = 0, ri = 0;
    for (int q = 0; q < 3; ++q) {
      if (wx[q] == 0.0) continue;
      const cpx<R> v = ec[(size_t)(cy0 + a) * nqc + cx0 + q];
      rr += wx[q] * (double)v.x;
      ri += wx[q] * (double)v.y;
    }
    sr += wy[a] * rr;
    si += wy[a] * ri;
  }
  return make_double2(sr, si);
}

constexpr int kLoads = (kE * kE + 255) / 256;

// Load the tile and halo of x (zero when xi is null), plus P ec when ec is
// given, into the parity sub-grids.  Boundary and outside nodes are zero.
template <typename R>
__device__ __forceinline__ void load_tile(cpx<R>* sx, const cpx<R>* __restrict__ xi, const cpx<R>* __restrict__ ec,
                                          int nq, int X0, int Y0) {
  cpx<R> v[kLoads];
#pragma unroll
  for (int i = 0; i < kLoads; ++i) {
    const int e = threadIdx.x + 256 * i;
    const int ey = e / kE, ex = e - ey * kE;
    const int gx = X0 - 2 + ex, gy = Y0 - 2 + ey;
    v[i] = cmk<cpx<R>>(0, 0);
    if (e < kE * kE && gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2) {
      if (xi) v[i] = xi[(size_t)gy * nq + gx];
      if (ec) {
        const double2 p = q2_prolong_at<R>(ec, (nq + 1) / 2, gx, gy);
        v[i] = cmk<cpx<R>>((double)v[i].x + p.x, (double)v[i].y + p.y);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kLoads; ++i) {
    const int e = threadIdx.x + 256 * i;
    if (e < kE * kE) {
      const int ey = e / kE, ex = e - ey * kE;
      sx[((ey & 1) * 2 + (ex & 1)) * kSub + (ey >> 1) * kH + (ex >> 1)] = v[i];
    }
  }
}

// One colour of the sweep for a lane of class (PX, PY).
template <int PX, int PY, bool CV, typename R>
__device__ __forceinline__ void sweep_node(cpx<R>* sx, int col, int la, int lb, int lane, int X0, int Y0, int nq,
                                           cpx<R> bv, const TCoef& t, const double* __restrict__ ctile) {
  int lx, ly;
  node_of<PX, PY>(col, la, lb, lx, ly);
  const int gx = X0 + lx, gy = Y0 + ly;
  if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) return;
  cpx<R>* base = sx + ((ly - PY) >> 1) * kH + ((lx - PX) >> 1);
  const double* cn = CV ? ctile + ((size_t)col * 64 + coff(PX, PY)) * 64 + lane : nullptr;
  double cd = 0;
  const double2 ax = stencil<PX, PY, CV, R>(base, cn, t, cd);
  double2 d = diag0<PX, PY>(t);
  if (CV) { d.x += t.er * cd; d.y += t.ei * cd; }
  const double er = (double)bv.x - ax.x, ei = (double)bv.y - ax.y;
  const double inv = 1.0 / (d.x * d.x + d.y * d.y);
  cpx<R>& xs = base[loff<PX, PY>(0, 0)];
  xs = cmk<cpx<R>>((double)xs.x + (er * d.x + ei * d.y) * inv, (double)xs.y + (ei * d.x - er * d.y) * inv);
}

template <int PX, int PY, typename R>
__device__ __forceinline__ void prefetch_b(cpx<R>* bb, const cpx<R>* __restrict__ bf, int la, int lb, int X0, int Y0,
                                           int nq) {
#pragma unroll
  for (int col = 0; col < 9; ++col) {
    int lx, ly;
    node_of<PX, PY>(col, la, lb, lx, ly);
    const int gx = X0 + lx, gy = Y0 + ly;
    bb[col] = (gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2) ? bf[(size_t)gy * nq + gx] : cmk<cpx<R>>(0, 0);
  }
}

// Write the tile interior from LDS (or zero on boundary nodes) to xo.
template <typename R>
__device__ __forceinline__ void store_tile(cpx<R>* __restrict__ xo, const cpx<R>* sx, int nq, int X0, int Y0) {
  for (int e = threadIdx.x; e < kT * kT; e += 256) {
    const int ly = e / kT, lx = e - ly * kT;
    const int gx = X0 + lx, gy = Y0 + ly;
    if (gx >= nq || gy >= nq) continue;
    const bool in = gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2;
    xo[(size_t)gy * nq + gx] =
        in ? sx[((ly & 1) * 2 + (lx & 1)) * kSub + ((ly + 2) >> 1) * kH + ((lx + 2) >> 1)] : cmk<cpx<R>>(0, 0);
  }
}

}  // namespace

// Sweep x -> xo.  xi == nullptr: start from x = 0.  ec != nullptr: start from
// x + P ec (coarse-grid correction of the V-cycle applied on load).
template <typename R, bool CV, bool FWD>
__global__ __launch_bounds__(256) void k_q2_sweep(cpx<R>* __restrict__ xo, const cpx<R>* __restrict__ xi,
                                                  const cpx<R>* __restrict__ b, const cpx<R>* __restrict__ ec, int n,
                                                  double h, const OpCoef* __restrict__ coef, int fpc,
                                                  const double* __restrict__ conv, int ntx, int nb, Mask mk) {
  __shared__ cpx<R> sx[4 * kSub];
  int tile, f;
  if (!tile_of_block(ntx * ntx, nb, CV, tile, f)) return;
  if (mk.off(f)) return;
  const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
  const int nq = 2 * n + 1, nqc = n + 1;
  const size_t off = (size_t)f * nq * nq;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, la = lane & 7, lb = lane >> 3;
  cpx<R> bb[9];
  switch (w) {
    case 0: prefetch_b<0, 0, R>(bb, b + off, la, lb, X0, Y0, nq); break;
    case 1: prefetch_b<1, 0, R>(bb, b + off, la, lb, X0, Y0, nq); break;
    case 2: prefetch_b<0, 1, R>(bb, b + off, la, lb, X0, Y0, nq); break;
    default: prefetch_b<1, 1, R>(bb, b + off, la, lb, X0, Y0, nq); break;
  }
  load_tile<R>(sx, xi ? xi + off : nullptr, ec ? ec + (size_t)f * nqc * nqc : nullptr, nq, X0, Y0);
  const TCoef t = tcoef(coef[f / fpc], h);
  const double* ctile = CV ? conv + (size_t)tile * 9 * 64 * 64 : nullptr;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int col = FWD ? k : 8 - k;
    switch (w) {
      case 0: sweep_node<0, 0, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, bb[col], t, ctile); break;
      case 1: sweep_node<1, 0, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, bb[col], t, ctile); break;
      case 2: sweep_node<0, 1, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, bb[col], t, ctile); break;
      default: sweep_node<1, 1, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, bb[col], t, ctile); break;
    }
    __syncthreads();
  }
  store_tile<R>(xo + off, sx, nq, X0, Y0);
}

namespace {
template <int PX, int PY, bool CV, typename R>
__device__ __forceinline__ double2 apply_node(const cpx<R>* sx, int col, int la, int lb, int lane, int X0, int Y0,
                                              int nq, const TCoef& t, const double* __restrict__ ctile) {
  int lx, ly;
  node_of<PX, PY>(col, la, lb, lx, ly);
  const int gx = X0 + lx, gy = Y0 + ly;
  if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) return make_double2(0, 0);
  const cpx<R>* base = sx + ((ly - PY) >> 1) * kH + ((lx - PX) >> 1);
  const double* cn = CV ? ctile + ((size_t)col * 64 + coff(PX, PY)) * 64 + lane : nullptr;
  double cd = 0;
  return stencil<PX, PY, CV, R>(base, cn, t, cd);
}

template <int PX, int PY>
__device__ __forceinline__ int stage_index(int col, int la, int lb) {
  int lx, ly;
  node_of<PX, PY>(col, la, lb, lx, ly);
  return ly * kT + lx;
}
}  // namespace

// out = b - A x (b != nullptr) or out = A x, on every node of the grids
// (zero on the boundary).  out and x must not alias.
template <typename R, bool CV>
__global__ __launch_bounds__(256) void k_q2_tile_apply(cpx<R>* __restrict__ out, const cpx<R>* __restrict__ x,
                                                       const cpx<R>* __restrict__ b, int n, double h,
                                                       const OpCoef* __restrict__ coef, int fpc,
                                                       const double* __restrict__ conv, int ntx, int nb, Mask mk) {
  __shared__ cpx<R> sx[4 * kSub];
  int tile, f;
  if (!tile_of_block(ntx * ntx, nb, CV, tile, f)) return;
  if (mk.off(f)) return;
  const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
  const int nq = 2 * n + 1;
  const size_t off = (size_t)f * nq * nq;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, la = lane & 7, lb = lane >> 3;
  load_tile<R>(sx, x + off, nullptr, nq, X0, Y0);
  const TCoef t = tcoef(coef[f / fpc], h);
  const double* ctile = CV ? conv + (size_t)tile * 9 * 64 * 64 : nullptr;
  __syncthreads();
  double2 acc[9];
#pragma unroll
  for (int col = 0; col < 9; ++col) {
    switch (w) {
      case 0: acc[col] = apply_node<0, 0, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, t, ctile); break;
      case 1: acc[col] = apply_node<1, 0, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, t, ctile); break;
      case 2: acc[col] = apply_node<0, 1, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, t, ctile); break;
      default: acc[col] = apply_node<1, 1, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, t, ctile); break;
    }
  }
  __syncthreads();
  // stage A x row-major (kT x kT) in the LDS tile for a coalesced store
#pragma unroll
  for (int col = 0; col < 9; ++col) {
    int i;
    switch (w) {
      case 0: i = stage_index<0, 0>(col, la, lb); break;
      case 1: i = stage_index<1, 0>(col, la, lb); break;
      case 2: i = stage_index<0, 1>(col, la, lb); break;
      default: i = stage_index<1, 1>(col, la, lb); break;
    }
    sx[i] = cmk<cpx<R>>(acc[col].x, acc[col].y);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kT * kT; e += 256) {
    const int ly = e / kT, lx = e - ly * kT;
    const int gx = X0 + lx, gy = Y0 + ly;
    if (gx >= nq || gy >= nq) continue;
    const size_t g = off + (size_t)gy * nq + gx;
    const bool in = gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2;
    cpx<R> v = in ? sx[e] : cmk<cpx<R>>(0, 0);
    if (b) v = in ? b[g] - v : cmk<cpx<R>>(0, 0);
    out[g] = v;
  }
}

// ------------------------------------------------------------ launchers
static inline unsigned tile_blocks(int ntx, int nb) {
  const unsigned total = (unsigned)(ntx * ntx) * (unsigned)nb;
  return (total + 7u) & ~7u;
}

int q2_tile_count(int n) {
  const int ntx = (2 * n + 1 + kT - 1) / kT;
  return ntx * ntx;
}

template <typename R>
void launch_q2_sweep(hipStream_t s, cpx<R>* xo, const cpx<R>* xi, const cpx<R>* b, const cpx<R>* ec, int n, double h,
                     const OpCoef* coef, int fpc, int nb, const double* tconv, bool forward, Mask mk) {
  const int ntx = (2 * n + 1 + kT - 1) / kT;
  const dim3 g(tile_blocks(ntx, nb)), blk(256);
  if (tconv) {
    if (forward) hipLaunchKernelGGL((k_q2_sweep<R, true, true>), g, blk, 0, s, xo, xi, b, ec, n, h, coef, fpc, tconv, ntx, nb, mk);
    else hipLaunchKernelGGL((k_q2_sweep<R, true, false>), g, blk, 0, s, xo, xi, b, ec, n, h, coef, fpc, tconv, ntx, nb, mk);
  } else {
    if (forward) hipLaunchKernelGGL((k_q2_sweep<R, false, true>), g, blk, 0, s, xo, xi, b, ec, n, h, coef, fpc, tconv, ntx, nb, mk);
    else hipLaunchKernelGGL((k_q2_sweep<R, false, false>), g, blk, 0, s, xo, xi, b, ec, n, h, coef, fpc, tconv, ntx, nb, mk);
  }
}

template <typename R>
void launch_q2_apply(hipStream_t s, cpx<R>* out, const cpx<R>* x, const cpx<R>* b, int n, double h,
                     const OpCoef* coef, int fpc, int nb, const double* tconv, Mask mk) {
  const int ntx = (2 * n + 1 + kT - 1) / kT;
  const dim3 g(tile_blocks(ntx, nb)), blk(256);
  if (tconv) hipLaunchKernelGGL((k_q2_tile_apply<R, true>), g, blk, 0, s, out, x, b, n, h, coef, fpc, tconv, ntx, nb, mk);
  else hipLaunchKernelGGL((k_q2_tile_apply<R, false>), g, blk, 0, s, out, x, b, n, h, coef, fpc, tconv, ntx, nb, mk);
}

// Reorder one half (0: N, 1: N^T) of a per-node convection table (50 values
// per padded Q2 node: 25 offsets of N, then 25 of N^T) into the layout of the
// tile kernels.
void q2_tile_conv_table(int n, const double* t50, int half, double* out) {
  const int nq = 2 * n + 1, ntx = (nq + kT - 1) / kT;
  const size_t total = (size_t)ntx * ntx * 9 * 64 * 64;
  for (size_t i = 0; i < total; ++i) out[i] = 0.0;
  for (int tile = 0; tile < ntx * ntx; ++tile) {
    const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
    for (int col = 0; col < 9; ++col) {
      const int cx = col % 3, cy = col / 3;
      for (int cls = 0; cls < 4; ++cls) {
        const int PX = cls & 1, PY = cls >> 1;
        for (int lane = 0; lane < 64; ++lane) {
          const int la = lane & 7, lb = lane >> 3;
          const int lx = cx + 3 * (2 * la + ((PX - cx) & 1)), ly = cy + 3 * (2 * lb + ((PY - cy) & 1));
          const int gx = X0 + lx, gy = Y0 + ly;
          if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) continue;
          int k = 0;
          for (int iy = 0; iy < wlen(PY); ++iy)
            for (int ix = 0; ix < wlen(PX); ++ix, ++k) {
              const int dx = wlo(PX) + ix, dy = wlo(PY) + iy;
              out[(((size_t)tile * 9 + col) * 64 + coff(PX, PY) + k) * 64 + lane] =
                  t50[((size_t)gy * nq + gx) * 50 + half * 25 + (dy + 2) * 5 + (dx + 2)];
            }
        }
      }
    }
  }
}

size_t q2_tile_conv_entries(int n) { return (size_t)q2_tile_count(n) * 9 * 64 * 64; }

#define PINTOC_Q2T_INST(R)                                                                                       \
  template void launch_q2_sweep<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, int, double, \
                                   const OpCoef*, int, int, const double*, bool, Mask);                             \
  template void launch_q2_apply<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, int, double, const OpCoef*,  \
                                   int, int, const double*, Mask);

PINTOC_Q2T_INST(double)
PINTOC_Q2T_INST(float)

}  // namespace pintoc
