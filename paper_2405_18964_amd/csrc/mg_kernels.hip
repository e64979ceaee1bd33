// Batched per-frequency kernels: scalar Q2/Q1 operators, multicolour
// Gauss-Seidel sweeps, residuals, grid transfers, coarsest-grid solves and
// Chebyshev steps (section 3.4: multigrid with SOR smoothing, Chebyshev
// semi-iteration for mass matrices).
//
// A "batch" is nb complex grids stored back to back.  Q2 grids are padded
// (2n+1)^2 with the Dirichlet boundary at zero; Q1 grids hold all (n+1)^2
// nodes (natural boundary conditions).  Grid f uses coefficient set
// coef[f / fpc] (fpc = grids per coefficient set).
#include "kernels.h"

namespace pintoc {

// Q2 operator  alpha M + gamma K + eta N + etat N^T  at interior node (ix, iy).
// Returns (A x)(ix, iy) and the diagonal entry.  The convection stencil table
// (if any) holds 25 coefficients per node for N and 25 for N^T.
template <typename R>
__device__ inline void q2_apply_node(const cpx<R>* __restrict__ x, int nq, int ix, int iy, double h,
                                     const OpCoef& c, const double* __restrict__ conv,
                                     cpx<R>& ax, cpx<R>& diag) {
  double mx[5], kx[5], my[5], ky[5];
  q2_rows(ix, h, mx, kx);
  q2_rows(iy, h, my, ky);
  // Offsets +-2 carry zero weight at midpoint nodes, which may sit next to the
  // boundary: clamp their indices so every load stays inside the grid.
  int cx[5], ry[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    cx[d] = min(max(ix + d - 2, 0), nq - 1);
    ry[d] = min(max(iy + d - 2, 0), nq - 1) * nq;
  }
  double amr = 0, ami = 0, akr = 0, aki = 0;   // M x and K x
#pragma unroll
  for (int dy = 0; dy < 5; ++dy) {
    double smr = 0, smi = 0, skr = 0, ski = 0;
#pragma unroll
    for (int dx = 0; dx < 5; ++dx) {
      cpx<R> v = x[ry[dy] + cx[dx]];
      smr += mx[dx] * (double)v.x; smi += mx[dx] * (double)v.y;
      skr += kx[dx] * (double)v.x; ski += kx[dx] * (double)v.y;
    }
    amr += my[dy] * smr; ami += my[dy] * smi;
    akr += ky[dy] * smr + my[dy] * skr; aki += ky[dy] * smi + my[dy] * ski;
  }
  double rr = c.alpha.x * amr - c.alpha.y * ami + c.gamma.x * akr - c.gamma.y * aki;
  double ri = c.alpha.x * ami + c.alpha.y * amr + c.gamma.x * aki + c.gamma.y * akr;
  const double md = mx[2] * my[2], kd = kx[2] * my[2] + mx[2] * ky[2];
  double dr = c.alpha.x * md + c.gamma.x * kd, di = c.alpha.y * md + c.gamma.y * kd;
  if (conv) {
    const double* cn = conv + (size_t)(iy * nq + ix) * 50;
    double nr = 0, ni = 0, tr = 0, ti = 0;
#pragma unroll
    for (int dy = 0; dy < 5; ++dy) {
#pragma unroll
      for (int dx = 0; dx < 5; ++dx) {
        cpx<R> v = x[ry[dy] + cx[dx]];
        const double a = cn[dy * 5 + dx], b = cn[25 + dy * 5 + dx];
        nr += a * (double)v.x; ni += a * (double)v.y;
        tr += b * (double)v.x; ti += b * (double)v.y;
      }
    }
    rr += c.eta.x * nr - c.eta.y * ni + c.etat.x * tr - c.etat.y * ti;
    ri += c.eta.x * ni + c.eta.y * nr + c.etat.x * ti + c.etat.y * tr;
    dr += c.eta.x * cn[12] + c.etat.x * cn[37];
    di += c.eta.y * cn[12] + c.etat.y * cn[37];
  }
  ax.x = (R)rr; ax.y = (R)ri;
  diag.x = (R)dr; diag.y = (R)di;
}

// Q1 operator on the unconstrained grid at node (ix, iy), 0 <= ix, iy <= n.
// Convection table: 9 coefficients per node for N and 9 for N^T.
template <typename R>
__device__ inline void q1_apply_node(const cpx<R>* __restrict__ x, int n, int ix, int iy, double h,
                                     const OpCoef& c, const double* __restrict__ conv,
                                     cpx<R>& ax, cpx<R>& diag) {
  const int np = n + 1;
  double mx[3], kx[3], my[3], ky[3];
  q1_rows(ix, n, h, mx, kx);
  q1_rows(iy, n, h, my, ky);
  double amr = 0, ami = 0, akr = 0, aki = 0;
  double nr = 0, ni = 0, tr = 0, ti = 0;
  const double* cn = conv ? conv + (size_t)(iy * np + ix) * 18 : nullptr;
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
    const int jy = iy + dy - 1;
    if (jy < 0 || jy > n) continue;
    double smr = 0, smi = 0, skr = 0, ski = 0;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int jx = ix + dx - 1;
      if (jx < 0 || jx > n) continue;
      cpx<R> v = x[jy * np + jx];
      smr += mx[dx] * (double)v.x; smi += mx[dx] * (double)v.y;
      skr += kx[dx] * (double)v.x; ski += kx[dx] * (double)v.y;
      if (cn) {
        const double a = cn[dy * 3 + dx], b = cn[9 + dy * 3 + dx];
        nr += a * (double)v.x; ni += a * (double)v.y;
        tr += b * (double)v.x; ti += b * (double)v.y;
      }
    }
    amr += my[dy] * smr; ami += my[dy] * smi;
    akr += ky[dy] * smr + my[dy] * skr; aki += ky[dy] * smi + my[dy] * ski;
  }
  double rr = c.alpha.x * amr - c.alpha.y * ami + c.gamma.x * akr - c.gamma.y * aki;
  double ri = c.alpha.x * ami + c.alpha.y * amr + c.gamma.x * aki + c.gamma.y * akr;
  const double md = mx[1] * my[1], kd = kx[1] * my[1] + mx[1] * ky[1];
  double dr = c.alpha.x * md + c.gamma.x * kd, di = c.alpha.y * md + c.gamma.y * kd;
  if (cn) {
    rr += c.eta.x * nr - c.eta.y * ni + c.etat.x * tr - c.etat.y * ti;
    ri += c.eta.x * ni + c.eta.y * nr + c.etat.x * ti + c.etat.y * tr;
    dr += c.eta.x * cn[4] + c.etat.x * cn[13];
    di += c.eta.y * cn[4] + c.etat.y * cn[13];
  }
  ax.x = (R)rr; ax.y = (R)ri;
  diag.x = (R)dr; diag.y = (R)di;
}

// (P e)(i, j) of the Q1 prolongation from the coarse grid (npc nodes per side):
// fine node i takes coarse i/2 (i even) or the mean of (i-1)/2 and (i+1)/2.
template <typename R>
__device__ inline double2 q1_prolong_at(const cpx<R>* __restrict__ ec, int npc, int i, int j) {
  const int ia = i >> 1, ib = (i + 1) >> 1, ja = j >> 1, jb = (j + 1) >> 1;
  const double wx = (i & 1) ? 0.5 : 1.0, wy = (j & 1) ? 0.5 : 1.0;
  const int nxs = (i & 1) ? 2 : 1, nys = (j & 1) ? 2 : 1;
  double sr = 0, si = 0;
  for (int a = 0; a < nys; ++a) {
    const int cy = a == 0 ? ja : jb;
    for (int q = 0; q < nxs; ++q) {
      const int cx = q == 0 ? ia : ib;
      const cpx<R> v = ec[(size_t)cy * npc + cx];
      sr += wx * wy * (double)v.x;
      si += wx * wy * (double)v.y;
    }
  }
  return make_double2(sr, si);
}

// ------------------------------------------------------ tiled GS sweeps
// Symmetric multicolour Gauss-Seidel inside square tiles, block Jacobi between
// tiles (a distributed SOR with one tile per subdomain).  A work-group owns
// one tile of one grid: it loads the tile and a halo into LDS, runs every
// colour in LDS (neighbour tiles keep the values the sweep started from), and
// writes the tile to xo.  xi and xo must be different buffers; xi == nullptr
// starts from x = 0, ec != nullptr adds the prolonged coarse correction P ec
// on load.  The Q2 sweep (and Q2 operator application) live in q2_tiles.hip.
constexpr int kT1 = 32, kL1 = kT1 + 2;       // Q1 tile and LDS side (halo 1)

template <typename R>
__global__ __launch_bounds__(256) void k_q1_tile_sweep(cpx<R>* __restrict__ xo, const cpx<R>* __restrict__ xi,
                                                       const cpx<R>* __restrict__ b, const cpx<R>* __restrict__ ec,
                                                       int n, double h,
                                                       const OpCoef* __restrict__ coef, int fpc,
                                                       const double* __restrict__ conv, int forward, int ntx, Mask mk) {
  __shared__ cpx<R> sx[kL1 * kL1];
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int X0 = (blockIdx.x % ntx) * kT1, Y0 = (blockIdx.x / ntx) * kT1;
  const int np = n + 1;
  const size_t off = (size_t)f * np * np;
  const int npc = n / 2 + 1;
  const cpx<R>* ecf = ec ? ec + (size_t)f * npc * npc : nullptr;
  for (int e = threadIdx.x; e < kL1 * kL1; e += blockDim.x) {
    const int gx = X0 - 1 + e % kL1, gy = Y0 - 1 + e / kL1;
    cpx<R> v = cmk<cpx<R>>(0, 0);
    if (gx >= 0 && gx <= n && gy >= 0 && gy <= n) {
      if (xi) v = xi[off + (size_t)gy * np + gx];
      if (ecf) {
        const double2 p = q1_prolong_at<R>(ecf, npc, gx, gy);
        v = cmk<cpx<R>>((double)v.x + p.x, (double)v.y + p.y);
      }
    }
    sx[e] = v;
  }
  const OpCoef c = coef[f / fpc];
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  for (int k = 0; k < 4; ++k) {
    const int col = forward ? k : 3 - k;
    const int lx = col % 2 + 2 * tx, ly = col / 2 + 2 * ty;
    const int gx = X0 + lx, gy = Y0 + ly;
    if (gx <= n && gy <= n) {
      double mx[3], kx[3], my[3], ky[3];
      q1_rows(gx, n, h, mx, kx);
      q1_rows(gy, n, h, my, ky);
      double amr = 0, ami = 0, akr = 0, aki = 0, nr = 0, ni = 0, tr = 0, ti = 0;
      const double* cn = conv ? conv + (size_t)(gy * np + gx) * 18 : nullptr;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        double smr = 0, smi = 0, skr = 0, ski = 0;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const cpx<R> v = sx[(ly + dy) * kL1 + lx + dx];
          smr += mx[dx] * (double)v.x; smi += mx[dx] * (double)v.y;
          skr += kx[dx] * (double)v.x; ski += kx[dx] * (double)v.y;
          if (cn) {
            const double a = cn[dy * 3 + dx], bb = cn[9 + dy * 3 + dx];
            nr += a * (double)v.x; ni += a * (double)v.y;
            tr += bb * (double)v.x; ti += bb * (double)v.y;
          }
        }
        amr += my[dy] * smr; ami += my[dy] * smi;
        akr += ky[dy] * smr + my[dy] * skr; aki += ky[dy] * smi + my[dy] * ski;
      }
      double rr = c.alpha.x * amr - c.alpha.y * ami + c.gamma.x * akr - c.gamma.y * aki;
      double ri = c.alpha.x * ami + c.alpha.y * amr + c.gamma.x * aki + c.gamma.y * akr;
      const double md = mx[1] * my[1], kd = kx[1] * my[1] + mx[1] * ky[1];
      double dr = c.alpha.x * md + c.gamma.x * kd, di = c.alpha.y * md + c.gamma.y * kd;
      if (cn) {
        rr += c.eta.x * nr - c.eta.y * ni + c.etat.x * tr - c.etat.y * ti;
        ri += c.eta.x * ni + c.eta.y * nr + c.etat.x * ti + c.etat.y * tr;
        dr += c.eta.x * cn[4] + c.etat.x * cn[13];
        di += c.eta.y * cn[4] + c.etat.y * cn[13];
      }
      const cpx<R> bi = b[off + (size_t)gy * np + gx];
      const double er = (double)bi.x - rr, ei = (double)bi.y - ri;
      const double den = dr * dr + di * di;
      cpx<R>& xs = sx[(ly + 1) * kL1 + lx + 1];
      xs = cmk<cpx<R>>((double)xs.x + (er * dr + ei * di) / den, (double)xs.y + (ei * dr - er * di) / den);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kT1 * kT1; e += blockDim.x) {
    const int gx = X0 + e % kT1, gy = Y0 + e / kT1;
    if (gx <= n && gy <= n) xo[off + (size_t)gy * np + gx] = sx[(e / kT1 + 1) * kL1 + e % kT1 + 1];
  }
}

// ------------------------------------------------------ residual r = b - A x
template <typename R>
__global__ __launch_bounds__(256) void k_q1_residual(cpx<R>* __restrict__ r, const cpx<R>* __restrict__ x, const cpx<R>* __restrict__ b,
                              int n, double h, const OpCoef* __restrict__ coef, int fpc,
                              const double* __restrict__ conv, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int np = n + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * np) return;
  const int ix = t % np, iy = t / np;
  cpx<R> ax, dg;
  q1_apply_node<R>(x + (size_t)f * np * np, n, ix, iy, h, coef[f / fpc], conv, ax, dg);
  const size_t i = (size_t)f * np * np + t;
  r[i] = b[i] - ax;
}

// y = A x (operator application; b = 0 residual form negated)
template <typename R>
__global__ __launch_bounds__(256) void k_q1_apply(cpx<R>* __restrict__ y, const cpx<R>* __restrict__ x, int n, double h,
                           const OpCoef* __restrict__ coef, int fpc, const double* __restrict__ conv, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int np = n + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * np) return;
  const int ix = t % np, iy = t / np;
  cpx<R> ax, dg;
  q1_apply_node<R>(x + (size_t)f * np * np, n, ix, iy, h, coef[f / fpc], conv, ax, dg);
  y[(size_t)f * np * np + t] = ax;
}

// ---------------------------------------------------------------- transfers
// (Q2 levels restrict inside k_q2_residual_restrict, q2_tiles.hip.)
// Q1: bc = P^T rf (coarse node I <-> fine 2I, weights 1/2, 1, 1/2).
template <typename R>
__global__ __launch_bounds__(256) void k_q1_restrict(cpx<R>* __restrict__ bc, const cpx<R>* __restrict__ rf, int nc, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int npc = nc + 1, nf = 2 * nc, npf = nf + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npc * npc) return;
  const int I = t % npc, J = t / npc;
  const cpx<R>* src = rf + (size_t)f * npf * npf;
  const double w[3] = {0.5, 1.0, 0.5};
  double sr = 0, si = 0;
  for (int dy = 0; dy < 3; ++dy) {
    const int fy = 2 * J + dy - 1;
    if (fy < 0 || fy > nf) continue;
    for (int dx = 0; dx < 3; ++dx) {
      const int fx = 2 * I + dx - 1;
      if (fx < 0 || fx > nf) continue;
      const cpx<R> v = src[(size_t)fy * npf + fx];
      sr += w[dx] * w[dy] * (double)v.x; si += w[dx] * w[dy] * (double)v.y;
    }
  }
  bc[(size_t)f * npc * npc + t] = cmk<cpx<R>>(sr, si);
}

// --------------------------------------------------------- coarsest grid
// N = 2 level.  Q2: 9 interior unknowns (padded 5x5 grid, nodes (1..3)^2);
// Q1: 9 nodes with node 0 held at zero and an 8x8 inverse for nodes 1..8.
// inv[ci] holds the dense inverse (row-major, complex FP64) per coefficient set.
template <typename R>
__global__ __launch_bounds__(256) void k_q2_coarse_solve(cpx<R>* __restrict__ x, const cpx<R>* __restrict__ b,
                                  const double2* __restrict__ inv, int fpc, int nb, Mask mk) {
  const int f = blockIdx.x * (blockDim.x / 9) + threadIdx.x / 9;
  const int r = threadIdx.x % 9;
  if (f >= nb || threadIdx.x >= (blockDim.x / 9) * 9 || mk.off(f)) return;
  const double2* A = inv + (size_t)(f / fpc) * 81;
  const cpx<R>* bb = b + (size_t)f * 25;
  double sr = 0, si = 0;
  for (int c = 0; c < 9; ++c) {
    const cpx<R> v = bb[(1 + c / 3) * 5 + 1 + c % 3];
    const double2 a = A[r * 9 + c];
    sr += a.x * (double)v.x - a.y * (double)v.y;
    si += a.x * (double)v.y + a.y * (double)v.x;
  }
  x[(size_t)f * 25 + (1 + r / 3) * 5 + 1 + r % 3] = cmk<cpx<R>>(sr, si);
}

template <typename R>
__global__ __launch_bounds__(256) void k_q1_coarse_solve(cpx<R>* __restrict__ x, const cpx<R>* __restrict__ b,
                                  const double2* __restrict__ inv, int fpc, int nb, Mask mk) {
  const int f = blockIdx.x * (blockDim.x / 9) + threadIdx.x / 9;
  const int r = threadIdx.x % 9;
  if (f >= nb || threadIdx.x >= (blockDim.x / 9) * 9 || mk.off(f)) return;
  if (r == 0) { x[(size_t)f * 9] = cmk<cpx<R>>(0, 0); return; }
  const double2* A = inv + (size_t)(f / fpc) * 64;
  const cpx<R>* bb = b + (size_t)f * 9;
  double sr = 0, si = 0;
  for (int c = 0; c < 8; ++c) {
    const cpx<R> v = bb[1 + c];
    const double2 a = A[(r - 1) * 8 + c];
    sr += a.x * (double)v.x - a.y * (double)v.y;
    si += a.x * (double)v.y + a.y * (double)v.x;
  }
  x[(size_t)f * 9 + r] = cmk<cpx<R>>(sr, si);
}

// ---------------------------------------------------------------- Chebyshev
// One step of the Jacobi-preconditioned Chebyshev semi-iteration for the
// mass matrix (Q2 interior or Q1 unconstrained):
//   first:  xn = g D^{-1} b
//   else:   xn = w (x - xp + g D^{-1}(b - M x)) + xp
// xn may alias xp (each thread reads its own xp entry before writing).
template <typename R>
__global__ __launch_bounds__(256) void k_q2_cheb(cpx<R>* xn, const cpx<R>* __restrict__ x, const cpx<R>* xp,
                          const cpx<R>* __restrict__ b, int n, double h, double g, double w, int first, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int nq = 2 * n + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nq * nq) return;
  const int ix = t % nq, iy = t / nq;
  const size_t i = (size_t)f * nq * nq + t;
  if (ix == 0 || iy == 0 || ix == nq - 1 || iy == nq - 1) { xn[i] = cmk<cpx<R>>(0, 0); return; }
  OpCoef c; c.alpha = make_double2(1, 0); c.gamma = make_double2(0, 0);
  c.eta = c.gamma; c.etat = c.gamma;
  if (first) {
    double mx[5], kx[5], my[5], ky[5];
    q2_rows(ix, h, mx, kx); q2_rows(iy, h, my, ky);
    const double d = mx[2] * my[2];
    const cpx<R> bi = b[i];
    xn[i] = cmk<cpx<R>>(g * (double)bi.x / d, g * (double)bi.y / d);
    return;
  }
  cpx<R> ax, dg;
  q2_apply_node<R>(x + (size_t)f * nq * nq, nq, ix, iy, h, c, nullptr, ax, dg);
  const cpx<R> bi = b[i], xi = x[i], pi = xp[i];
  const double d = (double)dg.x;
  xn[i] = cmk<cpx<R>>(w * ((double)xi.x - (double)pi.x + g * ((double)bi.x - (double)ax.x) / d) + (double)pi.x,
                      w * ((double)xi.y - (double)pi.y + g * ((double)bi.y - (double)ax.y) / d) + (double)pi.y);
}

template <typename R>
__global__ __launch_bounds__(256) void k_q1_cheb(cpx<R>* xn, const cpx<R>* __restrict__ x, const cpx<R>* xp,
                          const cpx<R>* __restrict__ b, int n, double h, double g, double w, int first, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int np = n + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * np) return;
  const int ix = t % np, iy = t / np;
  const size_t i = (size_t)f * np * np + t;
  OpCoef c; c.alpha = make_double2(1, 0); c.gamma = make_double2(0, 0);
  c.eta = c.gamma; c.etat = c.gamma;
  cpx<R> ax, dg;
  if (first) {
    double mx[3], kx[3], my[3], ky[3];
    q1_rows(ix, n, h, mx, kx); q1_rows(iy, n, h, my, ky);
    const double d = mx[1] * my[1];
    const cpx<R> bi = b[i];
    xn[i] = cmk<cpx<R>>(g * (double)bi.x / d, g * (double)bi.y / d);
    return;
  }
  q1_apply_node<R>(x + (size_t)f * np * np, n, ix, iy, h, c, nullptr, ax, dg);
  const cpx<R> bi = b[i], xi = x[i], pi = xp[i];
  const double d = (double)dg.x;
  xn[i] = cmk<cpx<R>>(w * ((double)xi.x - (double)pi.x + g * ((double)bi.x - (double)ax.x) / d) + (double)pi.x,
                      w * ((double)xi.y - (double)pi.y + g * ((double)bi.y - (double)ax.y) / d) + (double)pi.y);
}

// ------------------------------------------------ pressure pin in / pin out
// out = a_j yK + g_j yM, then shift by out[node 0] so that node 0 is zero
// (R (I - 1 e0^T)).  Coefficients per grid pair: ab[f / fpc] = (a, g) real.
template <typename R>
__global__ __launch_bounds__(256) void k_schur_combine_pin(cpx<R>* __restrict__ out, const cpx<R>* __restrict__ yK,
                                    const cpx<R>* __restrict__ yM, const double2* __restrict__ ab,
                                    int fpc, int nn, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nn) return;
  const double a = ab[f / fpc].x, g = ab[f / fpc].y;
  const size_t o = (size_t)f * nn;
  const cpx<R> k0 = yK[o], m0 = yM[o], k = yK[o + t], m = yM[o + t];
  out[o + t] = cmk<cpx<R>>(a * ((double)k.x - (double)k0.x) + g * ((double)m.x - (double)m0.x),
                           a * ((double)k.y - (double)k0.y) + g * ((double)m.y - (double)m0.y));
}

// ------------------------------------------------------------ launchers
static inline dim3 grid2(long work, int nb, int bs = 256) { return dim3((unsigned)((work + bs - 1) / bs), nb); }

template <typename R>
void launch_tile_sweep(hipStream_t s, bool q2, cpx<R>* xo, const cpx<R>* xi, const cpx<R>* b, const cpx<R>* ec,
                       int n, double h, const OpCoef* coef, int fpc, int nb, const double* conv, bool forward,
                       Mask mk) {
  if (q2) {
    launch_q2_sweep<R>(s, xo, xi, b, ec, n, h, coef, fpc, nb, conv, forward, mk);
  } else {
    const int np = n + 1, ntx = (np + kT1 - 1) / kT1;
    hipLaunchKernelGGL(k_q1_tile_sweep<R>, dim3(ntx * ntx, nb), dim3(256), 0, s, xo, xi, b, ec, n, h, coef, fpc,
                       conv, forward ? 1 : 0, ntx, mk);
  }
}

template <typename R>
void launch_q1_residual(hipStream_t s, cpx<R>* r, const cpx<R>* x, const cpx<R>* b, int n, double h,
                        const OpCoef* coef, int fpc, int nb, const double* conv, Mask mk) {
  const int np = n + 1;
  hipLaunchKernelGGL(k_q1_residual<R>, grid2((long)np * np, nb), dim3(256), 0, s, r, x, b, n, h, coef, fpc, conv, mk);
}

template <typename R>
void launch_apply(hipStream_t s, bool q2, cpx<R>* y, const cpx<R>* x, int n, double h, const OpCoef* coef,
                  int fpc, int nb, const double* conv, Mask mk) {
  if (q2) {
    launch_q2_apply<R>(s, y, x, nullptr, n, h, coef, fpc, nb, conv, mk);
  } else {
    const int np = n + 1;
    hipLaunchKernelGGL(k_q1_apply<R>, grid2((long)np * np, nb), dim3(256), 0, s, y, x, n, h, coef, fpc, conv, mk);
  }
}

template <typename R>
void launch_q1_restrict(hipStream_t s, cpx<R>* bc, const cpx<R>* rf, int nc, int nb, Mask mk) {
  const int npc = nc + 1;
  hipLaunchKernelGGL(k_q1_restrict<R>, grid2((long)npc * npc, nb), dim3(256), 0, s, bc, rf, nc, mk);
}

template <typename R>
void launch_coarse(hipStream_t s, bool q2, cpx<R>* x, const cpx<R>* b, const double2* inv, int fpc, int nb, Mask mk) {
  const int per = 256 / 9;
  const unsigned blocks = (unsigned)((nb + per - 1) / per);
  if (q2) hipLaunchKernelGGL(k_q2_coarse_solve<R>, dim3(blocks), dim3(256), 0, s, x, b, inv, fpc, nb, mk);
  else hipLaunchKernelGGL(k_q1_coarse_solve<R>, dim3(blocks), dim3(256), 0, s, x, b, inv, fpc, nb, mk);
}

template <typename R>
void launch_cheb(hipStream_t s, bool q2, cpx<R>* xn, const cpx<R>* x, const cpx<R>* xp, const cpx<R>* b, int n,
                 double h, double g, double w, int first, int nb, Mask mk) {
  if (q2) {
    const int nq = 2 * n + 1;
    hipLaunchKernelGGL(k_q2_cheb<R>, grid2((long)nq * nq, nb), dim3(256), 0, s, xn, x, xp, b, n, h, g, w, first, mk);
  } else {
    const int np = n + 1;
    hipLaunchKernelGGL(k_q1_cheb<R>, grid2((long)np * np, nb), dim3(256), 0, s, xn, x, xp, b, n, h, g, w, first, mk);
  }
}

template <typename R>
void launch_schur_combine_pin(hipStream_t s, cpx<R>* out, const cpx<R>* yK, const cpx<R>* yM, const double2* ab,
                              int fpc, int nn, int nb, Mask mk) {
  hipLaunchKernelGGL(k_schur_combine_pin<R>, grid2(nn, nb), dim3(256), 0, s, out, yK, yM, ab, fpc, nn, mk);
}

#define PINTOC_INST(R)                                                                                        \
  template void launch_tile_sweep<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, int, \
                                     double, const OpCoef*, int, int, const double*, bool, Mask);                    \
  template void launch_q1_residual<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, int, double,          \
                                      const OpCoef*, int, int, const double*, Mask);                                 \
  template void launch_apply<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, int, double, const OpCoef*, int, int, \
                                const double*, Mask);                                                                \
  template void launch_q1_restrict<R>(hipStream_t, cpx<R>*, const cpx<R>*, int, int, Mask);                          \
  template void launch_coarse<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, const double2*, int, int, Mask);         \
  template void launch_cheb<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, int,    \
                               double, double, double, int, int, Mask);                                              \
  template void launch_schur_combine_pin<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, const double2*, \
                                            int, int, int, Mask);

PINTOC_INST(double)
PINTOC_INST(float)

}  // namespace pintoc
