// Batched per-frequency kernels: scalar Q2/Q1 operators, multicolour
// Gauss-Seidel sweeps, residuals, grid transfers, coarsest-grid solves and
// Chebyshev steps (section 3.4: multigrid with SOR smoothing, Chebyshev
// semi-iteration for mass matrices).
//
// Arithmetic runs in the grids' precision R (stencil rows are formed in FP64
// and rounded once); the coarsest-grid solves accumulate in FP64.
//
// A "batch" is nb complex grids stored back to back.  Q2 grids are padded
// (2n+1)^2 with the Dirichlet boundary at zero; Q1 grids hold all (n+1)^2
// nodes (natural boundary conditions).  Grid f uses coefficient set
// coef[f / fpc] (fpc = grids per coefficient set).
#include "kernels.h"

namespace pintoc {

// 1-D stencil rows in precision R
template <typename R>
__device__ __forceinline__ void q2_rows_r(int i, double h, R m[5], R k[5]) {
  double md[5], kd[5];
  q2_rows(i, h, md, kd);
#pragma unroll
  for (int d = 0; d < 5; ++d) { m[d] = (R)md[d]; k[d] = (R)kd[d]; }
}
template <typename R>
__device__ __forceinline__ void q1_rows_r(int i, int n, double h, R m[3], R k[3]) {
  double md[3], kd[3];
  q1_rows(i, n, h, md, kd);
#pragma unroll
  for (int d = 0; d < 3; ++d) { m[d] = (R)md[d]; k[d] = (R)kd[d]; }
}

// Operator coefficients in precision R
template <typename R>
struct OpR {
  R ar, ai, gr, gi, er, ei, tr, ti;
  __device__ __forceinline__ explicit OpR(const OpCoef& c)
      : ar((R)c.alpha.x), ai((R)c.alpha.y), gr((R)c.gamma.x), gi((R)c.gamma.y), er((R)c.eta.x), ei((R)c.eta.y),
        tr((R)c.etat.x), ti((R)c.etat.y) {}
};

// Q2 operator  alpha M + gamma K + eta N + etat N^T  at interior node (ix, iy).
// Returns (A x)(ix, iy) and the diagonal entry.  The convection stencil table
// (if any) holds 25 coefficients per node for N and 25 for N^T.
template <typename R>
__device__ inline void q2_apply_node(const cpx<R>* __restrict__ x, int nq, int ix, int iy, double h,
                                     const OpCoef& c, const double* __restrict__ conv,
                                     cpx<R>& ax, cpx<R>& diag) {
  R mx[5], kx[5], my[5], ky[5];
  q2_rows_r<R>(ix, h, mx, kx);
  q2_rows_r<R>(iy, h, my, ky);
  const OpR<R> o(c);
  // Offsets +-2 carry zero weight at midpoint nodes, which may sit next to the
  // boundary: clamp their indices so every load stays inside the grid.
  int cx[5], ry[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    cx[d] = min(max(ix + d - 2, 0), nq - 1);
    ry[d] = min(max(iy + d - 2, 0), nq - 1) * nq;
  }
  R amr = 0, ami = 0, akr = 0, aki = 0;        // M x and K x
#pragma unroll
  for (int dy = 0; dy < 5; ++dy) {
    R smr = 0, smi = 0, skr = 0, ski = 0;
#pragma unroll
    for (int dx = 0; dx < 5; ++dx) {
      cpx<R> v = x[ry[dy] + cx[dx]];
      smr += mx[dx] * v.x; smi += mx[dx] * v.y;
      skr += kx[dx] * v.x; ski += kx[dx] * v.y;
    }
    amr += my[dy] * smr; ami += my[dy] * smi;
    akr += ky[dy] * smr + my[dy] * skr; aki += ky[dy] * smi + my[dy] * ski;
  }
  R rr = o.ar * amr - o.ai * ami + o.gr * akr - o.gi * aki;
  R ri = o.ar * ami + o.ai * amr + o.gr * aki + o.gi * akr;
  const R md = mx[2] * my[2], kd = kx[2] * my[2] + mx[2] * ky[2];
  R dr = o.ar * md + o.gr * kd, di = o.ai * md + o.gi * kd;
  if (conv) {
    const double* cn = conv + (size_t)(iy * nq + ix) * 50;
    R nr = 0, ni = 0, tr = 0, ti = 0;
#pragma unroll
    for (int dy = 0; dy < 5; ++dy) {
#pragma unroll
      for (int dx = 0; dx < 5; ++dx) {
        cpx<R> v = x[ry[dy] + cx[dx]];
        const R a = (R)cn[dy * 5 + dx], b = (R)cn[25 + dy * 5 + dx];
        nr += a * v.x; ni += a * v.y;
        tr += b * v.x; ti += b * v.y;
      }
    }
    rr += o.er * nr - o.ei * ni + o.tr * tr - o.ti * ti;
    ri += o.er * ni + o.ei * nr + o.tr * ti + o.ti * tr;
    dr += o.er * (R)cn[12] + o.tr * (R)cn[37];
    di += o.ei * (R)cn[12] + o.ti * (R)cn[37];
  }
  ax.x = rr; ax.y = ri;
  diag.x = dr; diag.y = di;
}

// Q1 operator on the unconstrained grid at node (ix, iy), 0 <= ix, iy <= n.
// Convection table: 9 coefficients per node for N and 9 for N^T.
template <typename R>
__device__ inline void q1_apply_node(const cpx<R>* __restrict__ x, int n, int ix, int iy, double h,
                                     const OpCoef& c, const double* __restrict__ conv,
                                     cpx<R>& ax, cpx<R>& diag) {
  const int np = n + 1;
  R mx[3], kx[3], my[3], ky[3];
  q1_rows_r<R>(ix, n, h, mx, kx);
  q1_rows_r<R>(iy, n, h, my, ky);
  const OpR<R> o(c);
  R amr = 0, ami = 0, akr = 0, aki = 0;
  R nr = 0, ni = 0, tr = 0, ti = 0;
  const double* cn = conv ? conv + (size_t)(iy * np + ix) * 18 : nullptr;
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
    const int jy = iy + dy - 1;
    if (jy < 0 || jy > n) continue;
    R smr = 0, smi = 0, skr = 0, ski = 0;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int jx = ix + dx - 1;
      if (jx < 0 || jx > n) continue;
      cpx<R> v = x[jy * np + jx];
      smr += mx[dx] * v.x; smi += mx[dx] * v.y;
      skr += kx[dx] * v.x; ski += kx[dx] * v.y;
      if (cn) {
        const R a = (R)cn[dy * 3 + dx], b = (R)cn[9 + dy * 3 + dx];
        nr += a * v.x; ni += a * v.y;
        tr += b * v.x; ti += b * v.y;
      }
    }
    amr += my[dy] * smr; ami += my[dy] * smi;
    akr += ky[dy] * smr + my[dy] * skr; aki += ky[dy] * smi + my[dy] * ski;
  }
  R rr = o.ar * amr - o.ai * ami + o.gr * akr - o.gi * aki;
  R ri = o.ar * ami + o.ai * amr + o.gr * aki + o.gi * akr;
  const R md = mx[1] * my[1], kd = kx[1] * my[1] + mx[1] * ky[1];
  R dr = o.ar * md + o.gr * kd, di = o.ai * md + o.gi * kd;
  if (cn) {
    rr += o.er * nr - o.ei * ni + o.tr * tr - o.ti * ti;
    ri += o.er * ni + o.ei * nr + o.tr * ti + o.ti * tr;
    dr += o.er * (R)cn[4] + o.tr * (R)cn[13];
    di += o.ei * (R)cn[4] + o.ti * (R)cn[13];
  }
  ax.x = rr; ax.y = ri;
  diag.x = dr; diag.y = di;
}

// (P e)(i, j) of the Q1 prolongation from the coarse grid (npc nodes per side):
// fine node i takes coarse i/2 (i even) or the mean of (i-1)/2 and (i+1)/2.
template <typename R>
__device__ inline cpx<R> q1_prolong_at(const cpx<R>* __restrict__ ec, int npc, int i, int j) {
  const int ia = i >> 1, ib = (i + 1) >> 1, ja = j >> 1, jb = (j + 1) >> 1;
  const R wx = (i & 1) ? R(0.5) : R(1), wy = (j & 1) ? R(0.5) : R(1);
  const int nxs = (i & 1) ? 2 : 1, nys = (j & 1) ? 2 : 1;
  cpx<R> s = cmk<cpx<R>>(0, 0);
  for (int a = 0; a < nys; ++a) {
    const int cy = a == 0 ? ja : jb;
    for (int q = 0; q < nxs; ++q) {
      const int cx = q == 0 ? ia : ib;
      const cpx<R> v = ec[(size_t)cy * npc + cx];
      s.x += wx * wy * v.x;
      s.y += wx * wy * v.y;
    }
  }
  return s;
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
        const cpx<R> p = q1_prolong_at<R>(ecf, npc, gx, gy);
        v.x += p.x;
        v.y += p.y;
      }
    }
    sx[e] = v;
  }
  const OpR<R> o(coef[f / fpc]);
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  for (int k = 0; k < 4; ++k) {
    const int col = forward ? k : 3 - k;
    const int lx = col % 2 + 2 * tx, ly = col / 2 + 2 * ty;
    const int gx = X0 + lx, gy = Y0 + ly;
    if (gx <= n && gy <= n) {
      R mx[3], kx[3], my[3], ky[3];
      q1_rows_r<R>(gx, n, h, mx, kx);
      q1_rows_r<R>(gy, n, h, my, ky);
      R amr = 0, ami = 0, akr = 0, aki = 0, nr = 0, ni = 0, tr = 0, ti = 0;
      const double* cn = conv ? conv + (size_t)(gy * np + gx) * 18 : nullptr;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        R smr = 0, smi = 0, skr = 0, ski = 0;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const cpx<R> v = sx[(ly + dy) * kL1 + lx + dx];
          smr += mx[dx] * v.x; smi += mx[dx] * v.y;
          skr += kx[dx] * v.x; ski += kx[dx] * v.y;
          if (cn) {
            const R a = (R)cn[dy * 3 + dx], bb = (R)cn[9 + dy * 3 + dx];
            nr += a * v.x; ni += a * v.y;
            tr += bb * v.x; ti += bb * v.y;
          }
        }
        amr += my[dy] * smr; ami += my[dy] * smi;
        akr += ky[dy] * smr + my[dy] * skr; aki += ky[dy] * smi + my[dy] * ski;
      }
      R rr = o.ar * amr - o.ai * ami + o.gr * akr - o.gi * aki;
      R ri = o.ar * ami + o.ai * amr + o.gr * aki + o.gi * akr;
      const R md = mx[1] * my[1], kd = kx[1] * my[1] + mx[1] * ky[1];
      R dr = o.ar * md + o.gr * kd, di = o.ai * md + o.gi * kd;
      if (cn) {
        rr += o.er * nr - o.ei * ni + o.tr * tr - o.ti * ti;
        ri += o.er * ni + o.ei * nr + o.tr * ti + o.ti * tr;
        dr += o.er * (R)cn[4] + o.tr * (R)cn[13];
        di += o.ei * (R)cn[4] + o.ti * (R)cn[13];
      }
      const cpx<R> bi = b[off + (size_t)gy * np + gx];
      const R er = bi.x - rr, ei = bi.y - ri;
      const R den = dr * dr + di * di;
      cpx<R>& xs = sx[(ly + 1) * kL1 + lx + 1];
      cpx<R> nxv;
      nxv.x = xs.x + (er * dr + ei * di) / den;
      nxv.y = xs.y + (ei * dr - er * di) / den;
      xs = nxv;
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
  const R w[3] = {R(0.5), R(1), R(0.5)};
  cpx<R> sv = cmk<cpx<R>>(0, 0);
  for (int dy = 0; dy < 3; ++dy) {
    const int fy = 2 * J + dy - 1;
    if (fy < 0 || fy > nf) continue;
    for (int dx = 0; dx < 3; ++dx) {
      const int fx = 2 * I + dx - 1;
      if (fx < 0 || fx > nf) continue;
      const cpx<R> v = src[(size_t)fy * npf + fx];
      sv.x += w[dx] * w[dy] * v.x; sv.y += w[dx] * w[dy] * v.y;
    }
  }
  bc[(size_t)f * npc * npc + t] = sv;
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

// ------------------------------------------------ small-grid V-cycles
// The rest of a Q2 V(1,1) cycle from level n0 <= kSmallN down to the N = 2
// grid in one work-group per grid with every level in LDS.  With convection
// the operator gains eta C, C read from a per-node table of the levels
// n0 .. 4 (q2_small_conv_table; the coarsest inverse already holds it).  A
// 48-node tile covers these grids, so the tiled smoother is plain
// multicolour Gauss-Seidel (colour 3 (gy % 3) + gx % 3, forward before and
// backward after the coarse correction; L lanes share a node's stencil rows
// and add their parts before the update); residual,
// restriction P^T, exact coarsest solve (FP64 accumulation, as in
// k_q2_coarse_solve) and prolongation P follow the per-level kernels.
// x0 == nullptr: the cycle starts from zero on level n0; x0 may equal xg
// (every grid is read into LDS before it is written back).
constexpr int kSmallN = kQ2SmallN;

namespace {
constexpr int sq(int v) { return v * v; }
constexpr int kSmallEntries = sq(2 * kSmallN + 1) + sq(kSmallN + 1) + sq(kSmallN / 2 + 1) + sq(kSmallN / 4 + 1);
// waves per work-group for L lanes per colour slot
template <int L> constexpr int kSmallWaves = L == 4 ? 8 : 4;
static_assert(4 * sq((2 * kSmallN + 3) / 3) <= 512, "four lanes per colour slot in a 512-thread work-group");
static_assert(sq((2 * kSmallN + 3) / 3) <= 256, "one lane per colour slot in a 256-thread work-group");

// m' . v and k' . v along one direction for node parity P (offsets -2..2 or -1..1)
template <typename R>
__device__ __forceinline__ void small_comb(int P, const R* v, R& m, R& k) {
  if (P == 0) {
    const R s04 = v[0] + v[4], s13 = v[1] + v[3];
    m = R(8) * v[2] + R(2) * s13 - s04;
    k = R(14) * v[2] - R(8) * s13 + s04;
  } else {
    const R s02 = v[1] + v[3];
    m = R(16) * v[2] + R(2) * s02;
    k = R(16) * v[2] - R(8) * s02;
  }
}

// Level operator coefficients: integer-weight scales of M and K, eta of the
// convection table tl (level table of q2_small_conv_table, or null)
template <typename R>
struct SmallOp {
  R ar, ai, gr, gi, er, ei;
  const R* tl;
  int per;                                            // nodes per colour and direction
};

template <typename R>
__device__ __forceinline__ SmallOp<R> small_op(const OpCoef& c, int n, const R* tl) {
  const double h = 1.0 / n, sm = h * h / 900.0;
  return SmallOp<R>{(R)(c.alpha.x * sm), (R)(c.alpha.y * sm), (R)(c.gamma.x / 90.0), (R)(c.gamma.y / 90.0),
                    (R)c.eta.x, (R)c.eta.y, tl, (2 * n + 3) / 3};
}

// 1-D weights m'(d), k'(d) (offset d - 2) of a node of parity P: the rows
// that small_comb applies
template <typename R>
__device__ __forceinline__ R small_mw(int P, int d) {
  if (d == 2) return P ? R(16) : R(8);
  if (d == 1 || d == 3) return R(2);
  return P ? R(0) : R(-1);
}
template <typename R>
__device__ __forceinline__ R small_kw(int P, int d) {
  if (d == 2) return P ? R(16) : R(14);
  if (d == 1 || d == 3) return R(-8);
  return P ? R(0) : R(1);
}

// Rows of the 5 x 5 stencil window handled by lane q of the L lanes that
// share a node: dy = q, q + L, .. (at most kRows(L) of them).
template <int L> constexpr int kRows = (5 + L - 1) / L;

// the convection coefficients of lane q's rows at slot e of colour col (zero
// outside the grid): tv[5 r + dx] for row dy = q + r L
template <typename R, int L>
__device__ __forceinline__ void small_tab(const SmallOp<R>& o, int col, int e, int q, R* tv) {
  const int pp = o.per * o.per;
  const R* t = o.tl + (size_t)col * 25 * pp + e;
#pragma unroll
  for (int r = 0; r < kRows<L>; ++r) {
    const int dy = q + r * L;
    if (dy < 5) {
#pragma unroll
      for (int dx = 0; dx < 5; ++dx) tv[5 * r + dx] = t[(5 * dy + dx) * pp];
    }
  }
}

// Lane q's share of (A x)(gx, gy) for alpha M + gamma K (+ eta C, with the
// lane's coefficients tv) on a padded grid in LDS: the rows dy = q + r L of
// the window, weighted by their 1-D y-weights, and (CV) the lane's part of
// the diagonal convection entry.  Summed over the L lanes this is A x.
// Offsets +-2 of a midpoint node carry no weight in M, K or C.
template <typename R, bool CV, int L>
__device__ __forceinline__ void small_apply(const cpx<R>* x, int nq, int gx, int gy, int q, const SmallOp<R>& o,
                                            const R* tv, R& axr, R& axi, R& cdg) {
  const int px = gx & 1, py = gy & 1;
  R pmr = 0, pmi = 0, pkr = 0, pki = 0, cr = 0, ci = 0;
  cdg = 0;
#pragma unroll
  for (int r = 0; r < kRows<L>; ++r) {
    const int dy = q + r * L;
    if (dy >= 5 || (py && (dy == 0 || dy == 4))) continue;
    R vr[5], vi[5];
#pragma unroll
    for (int dx = 0; dx < 5; ++dx) {
      const bool u = px == 0 || (dx >= 1 && dx <= 3);
      const cpx<R> v = u ? x[(gy + dy - 2) * nq + gx + dx - 2] : cmk<cpx<R>>(0, 0);
      vr[dx] = v.x;
      vi[dx] = v.y;
      if (CV) {
        cr += tv[5 * r + dx] * v.x;
        ci += tv[5 * r + dx] * v.y;
      }
    }
    R smr, skr, smi, ski;
    small_comb<R>(px, vr, smr, skr);
    small_comb<R>(px, vi, smi, ski);
    const R wm = small_mw<R>(py, dy), wk = small_kw<R>(py, dy);
    pmr += wm * smr;                       // m'_y m'_x
    pmi += wm * smi;
    pkr += wk * smr + wm * skr;            // k'_y m'_x + m'_y k'_x
    pki += wk * smi + wm * ski;
    if (CV && dy == 2) cdg = tv[5 * r + 2];
  }
  axr = o.ar * pmr - o.ai * pmi + o.gr * pkr - o.gi * pki;
  axi = o.ar * pmi + o.ai * pmr + o.gr * pki + o.gi * pkr;
  if (CV) {
    axr += o.er * cr - o.ei * ci;
    axi += o.er * ci + o.ei * cr;
  }
}

// the diagonal of alpha M + gamma K + eta C at a node of parity (px, py)
// with diagonal convection entry cdg
template <typename R, bool CV>
__device__ __forceinline__ cpx<R> small_diag(const SmallOp<R>& o, int px, int py, R cdg) {
  const R md = (px ? R(16) : R(8)) * (py ? R(16) : R(8));
  const R kd = (px ? R(16) : R(14)) * (py ? R(16) : R(8)) + (px ? R(16) : R(8)) * (py ? R(16) : R(14));
  cpx<R> dg;
  dg.x = o.ar * md + o.gr * kd + (CV ? o.er * cdg : R(0));
  dg.y = o.ai * md + o.gi * kd + (CV ? o.ei * cdg : R(0));
  return dg;
}

// Sum over the 4 lanes of a quad (lanes 4i .. 4i + 3) by DPP quad
// permutations; every lane of the quad must be active.
template <int C>
__device__ __forceinline__ int dpp_i(int v) { return __builtin_amdgcn_update_dpp(0, v, C, 0xF, 0xF, true); }
template <int C>
__device__ __forceinline__ float dpp_r(float v) { return __int_as_float(dpp_i<C>(__float_as_int(v))); }
template <int C>
__device__ __forceinline__ double dpp_r(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<C>((int)(unsigned)(b & 0xffffffffll)), hi = dpp_i<C>((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename R, int L>
__device__ __forceinline__ R lane_sum(R v) {
  static_assert(L == 1 || L == 4, "lanes per node");
  if (L == 4) {
    v += dpp_r<0xB1>(v);                   // quad_perm [1, 0, 3, 2]
    v += dpp_r<0x4E>(v);                   // quad_perm [2, 3, 0, 1]
  }
  return v;
}

// one Gauss-Seidel sweep (forward or backward colour order) of level grid x.
// Lanes L s .. L s + L - 1 own slot s of every colour (per^2 L <= blockDim.x
// for n <= 16); their convection coefficients for the next colour are loaded
// while the current colour is updated.  Every thread reaches the lane sums.
template <typename R, bool CV, int L>
__device__ __forceinline__ void small_sweep(cpx<R>* x, const cpx<R>* b, int n, const SmallOp<R>& o, bool forward) {
  const int nq = 2 * n + 1, per = o.per, e = threadIdx.x / L, q = threadIdx.x % L;
  const bool mine = e < per * per;
  constexpr int kTv = 5 * kRows<L>;
  R cur[kTv], nxt[kTv];
  if (CV && mine) small_tab<R, L>(o, forward ? 0 : 8, e, q, cur);
  for (int k = 0; k < 9; ++k) {
    const int col = forward ? k : 8 - k, cx = col % 3, cy = col / 3;
    if (CV && mine && k < 8) small_tab<R, L>(o, forward ? col + 1 : col - 1, e, q, nxt);
    const int gx = cx + 3 * (e % per), gy = cy + 3 * (e / per);
    const bool act = mine && gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2;
    R axr = 0, axi = 0, cdg = 0;
    if (act) small_apply<R, CV, L>(x, nq, gx, gy, q, o, cur, axr, axi, cdg);
    axr = lane_sum<R, L>(axr);
    axi = lane_sum<R, L>(axi);
    if (CV) cdg = lane_sum<R, L>(cdg);
    if (act && q == 0) {
      const cpx<R> dg = small_diag<R, CV>(o, gx & 1, gy & 1, cdg);
      const cpx<R> bv = b[gy * nq + gx];
      const R er = bv.x - axr, ei = bv.y - axi, inv = R(1) / (dg.x * dg.x + dg.y * dg.y);
      cpx<R>& xs = x[gy * nq + gx];
      cpx<R> nv;
      nv.x = xs.x + (er * dg.x + ei * dg.y) * inv;
      nv.y = xs.y + (ei * dg.x - er * dg.y) * inv;
      xs = nv;
    }
    if (CV) {
#pragma unroll
      for (int i = 0; i < kTv; ++i) cur[i] = nxt[i];
    }
    __syncthreads();
  }
}

// 1-D weight of fine offset d (-3..3) in the restriction to a coarse node of parity P
template <typename R>
__device__ __forceinline__ R small_rw(int P, int d) {
  if (P) return d == 0 ? R(1) : ((d == 1 || d == -1) ? R(0.75) : R(0));
  return d == 0 ? R(1) : ((d == 1 || d == -1) ? R(0.375) : ((d == 3 || d == -3) ? R(-0.125) : R(0)));
}

// 1-D prolongation weight of coarse node 2e + q for fine node 4e + r
template <typename R>
__device__ __forceinline__ R small_pw(int r, int q) {
  if (r == 0) return q == 0 ? R(1) : R(0);
  if (r == 2) return q == 1 ? R(1) : R(0);
  if (r == 1) return q == 0 ? R(0.375) : (q == 1 ? R(0.75) : R(-0.125));
  return q == 0 ? R(-0.125) : (q == 1 ? R(0.75) : R(0.375));
}
}  // namespace

template <typename R, bool CV, int L>
__global__ __launch_bounds__(64 * kSmallWaves<L>) void k_q2_small_vcycle(cpx<R>* xg, const cpx<R>* x0,
                                                         const cpx<R>* __restrict__ bg, int n0,
                                                         const OpCoef* __restrict__ coef, int cstride, int fpc,
                                                         const double2* __restrict__ inv,
                                                         const R* __restrict__ tconv, int nb, Mask mk) {
  // x of every level and b of the coarser levels in LDS (the top level's b is
  // read from memory: 47.5 KB in FP64, three work-groups per CU)
  constexpr int kB = kSmallEntries - sq(2 * kSmallN + 1);
  __shared__ cpx<R> xs[kSmallEntries], bsc[kB], rs[sq(2 * kSmallN + 1)];
  const int f = blockIdx.x;
  if (f >= nb || mk.off(f)) return;
  int lev = 0, off[8], nn[8], toff[8];
  for (int n = n0, o = 0, t = 0; n >= 2; n >>= 1, ++lev) {
    off[lev] = o; nn[lev] = n; toff[lev] = t;
    o += sq(2 * n + 1);
    t += 225 * sq((2 * n + 3) / 3);
  }
  // level l's coefficients: coef[l cstride + set]
  auto op = [&](int l) {
    return small_op<R>(coef[(size_t)l * cstride + f / fpc], nn[l], CV ? tconv + toff[l] : nullptr);
  };
  const int nq0 = 2 * n0 + 1;
  const size_t g0 = (size_t)f * nq0 * nq0;
  const cpx<R>* b0 = bg + g0;
  // b of level l: level 0 in memory, level l >= 1 in LDS at off[l] - off[1]
  auto blev = [&](int l) -> const cpx<R>* { return l == 0 ? b0 : bsc + (off[l] - off[1]); };
  for (int e = threadIdx.x; e < nq0 * nq0; e += blockDim.x) xs[e] = x0 ? x0[g0 + e] : cmk<cpx<R>>(0, 0);
  for (int e = nq0 * nq0 + threadIdx.x; e < off[lev - 1] + 25; e += blockDim.x) xs[e] = cmk<cpx<R>>(0, 0);
  __syncthreads();
  // down: pre-smoothing, residual, restriction
  for (int l = 0; l + 1 < lev; ++l) {
    const int n = nn[l], nq = 2 * n + 1, nqc = n + 1;
    cpx<R>* x = xs + off[l];
    const cpx<R>* b = blev(l);
    const SmallOp<R> o = op(l);
    small_sweep<R, CV, L>(x, b, n, o, true);
    // residual over the colour slots (the convection table's order)
    const int pp = o.per * o.per;
    for (int i = threadIdx.x; i < 9 * pp; i += blockDim.x) {
      const int col = i / pp, e = i - col * pp;
      const int gx = col % 3 + 3 * (e % o.per), gy = col / 3 + 3 * (e / o.per);
      if (gx >= nq || gy >= nq) continue;
      cpx<R> r = cmk<cpx<R>>(0, 0);
      if (gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2) {
        R tv[25], axr, axi, cdg;
        if (CV) small_tab<R, 1>(o, col, e, 0, tv);
        small_apply<R, CV, 1>(x, nq, gx, gy, 0, o, tv, axr, axi, cdg);
        const cpx<R> bv = b[gy * nq + gx];
        r.x = bv.x - axr;
        r.y = bv.y - axi;
      }
      rs[gy * nq + gx] = r;
    }
    __syncthreads();
    cpx<R>* bc = bsc + (off[l + 1] - off[1]);
    for (int e = threadIdx.x; e < nqc * nqc; e += blockDim.x) {
      const int I = e % nqc, J = e / nqc;
      cpx<R> v = cmk<cpx<R>>(0, 0);
      if (I >= 1 && I <= nqc - 2 && J >= 1 && J <= nqc - 2) {
        for (int dy = -3; dy <= 3; ++dy) {
          const R wy = small_rw<R>(J & 1, dy);
          if (wy == R(0)) continue;
          R rr = 0, ri = 0;
          for (int dx = -3; dx <= 3; ++dx) {
            const R wx = small_rw<R>(I & 1, dx);
            if (wx == R(0)) continue;
            const cpx<R> rv = rs[(2 * J + dy) * nq + 2 * I + dx];
            rr += wx * rv.x;
            ri += wx * rv.y;
          }
          v.x += wy * rr;
          v.y += wy * ri;
        }
      }
      bc[e] = v;
    }
    __syncthreads();
  }
  // coarsest grid (N = 2): 9 interior unknowns of the padded 5 x 5 grid
  {
    const cpx<R>* b = blev(lev - 1);
    cpx<R>* x = xs + off[lev - 1];
    const double2* A = inv + (size_t)(f / fpc) * 81;
    if (threadIdx.x < 9) {
      const int r = threadIdx.x;
      double sr = 0, si = 0;
      for (int q = 0; q < 9; ++q) {
        const cpx<R> v = b[(1 + q / 3) * 5 + 1 + q % 3];
        const double2 a = A[r * 9 + q];
        sr += a.x * (double)v.x - a.y * (double)v.y;
        si += a.x * (double)v.y + a.y * (double)v.x;
      }
      x[(1 + r / 3) * 5 + 1 + r % 3] = cmk<cpx<R>>(sr, si);
    }
    __syncthreads();
  }
  // up: prolongation of the coarse correction, post-smoothing
  for (int l = lev - 2; l >= 0; --l) {
    const int n = nn[l], nq = 2 * n + 1, nqc = n + 1;
    cpx<R>* x = xs + off[l];
    const cpx<R>* ec = xs + off[l + 1];
    for (int e = threadIdx.x; e < nq * nq; e += blockDim.x) {
      const int gx = e % nq, gy = e / nq;
      if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) continue;
      const int ex = gx >> 2, rx = gx & 3, ey = gy >> 2, ry = gy & 3;
      R pr = 0, pi = 0;
      for (int qy = 0; qy < 3; ++qy) {
        const R wy = small_pw<R>(ry, qy);
        if (wy == R(0)) continue;
        for (int qx = 0; qx < 3; ++qx) {
          const R wx = small_pw<R>(rx, qx);
          if (wx == R(0)) continue;
          const cpx<R> v = ec[(2 * ey + qy) * nqc + 2 * ex + qx];
          pr += wy * (wx * v.x);
          pi += wy * (wx * v.y);
        }
      }
      x[e].x += pr;
      x[e].y += pi;
    }
    __syncthreads();
    small_sweep<R, CV, L>(x, blev(l), n, op(l), false);
  }
  for (int e = threadIdx.x; e < nq0 * nq0; e += blockDim.x) xg[g0 + e] = xs[e];
}

// lanes per colour slot of the small Q2 V-cycle: four (512 threads) with
// convection, where a node's stencil is the longest chain of a colour step,
// and in FP32, where four 512-thread work-groups still fit a CU; one for FP64
// without convection (its registers would leave two work-groups per CU)
template <typename R>
static int small_lanes(bool cv) { return (cv || sizeof(R) == 4) ? 4 : 1; }

template <typename R>
void launch_q2_small_vcycle(hipStream_t s, cpx<R>* x, const cpx<R>* x0, const cpx<R>* b, int n0, const OpCoef* coef,
                            int cstride, int fpc, const double2* inv, const R* tconv, int nb, Mask mk) {
  const dim3 g((unsigned)nb);
  const bool cv = tconv != nullptr;
  const int L = small_lanes<R>(cv);
#define PINTOC_SMALL(CV, LL)                                                                                       \
  if (cv == CV && L == LL) {                                                                                      \
    hipLaunchKernelGGL((k_q2_small_vcycle<R, CV, LL>), g, dim3(64 * kSmallWaves<LL>), 0, s, x, x0, b, n0, coef,    \
                       cstride, fpc, inv, tconv, nb, mk);                                                         \
    return;                                                                                                       \
  }
  PINTOC_SMALL(true, 4)
  PINTOC_SMALL(false, 1)
  PINTOC_SMALL(true, 1)
  PINTOC_SMALL(false, 4)
#undef PINTOC_SMALL
}

// Convection table of the small levels n0, n0 / 2, .., 4 for one operator
// half (0: N, 1: N^T), the levels back to back, in the order the small
// V-cycle's threads read it.  On a level (nq = 2n + 1, per = (nq + 2) / 3
// nodes per colour and direction) node (gx, gy) = (cx + 3 i, cy + 3 j) of
// colour col = 3 cy + cx is slot e = per j + i, and its coefficient of offset
// (dx, dy) in -2..2 sits at [(25 col + 5 (dy + 2) + dx + 2) per^2 + e]; slots
// off the interior hold zeros.  tabs[l] is level l's table of 50 values per
// padded node (N, then N^T).
size_t q2_small_conv_entries(int n0) {
  size_t e = 0;
  for (int n = n0; n >= 4; n >>= 1) e += (size_t)225 * ((2 * n + 3) / 3) * ((2 * n + 3) / 3);
  return e;
}

void q2_small_conv_table(int n0, const std::vector<const double*>& tabs, int half, double* out) {
  size_t base = 0;
  int l = 0;
  for (int n = n0; n >= 4; n >>= 1, ++l) {
    const int nq = 2 * n + 1, per = (nq + 2) / 3, pp = per * per;
    for (int col = 0; col < 9; ++col)
      for (int e = 0; e < pp; ++e) {
        const int gx = col % 3 + 3 * (e % per), gy = col / 3 + 3 * (e / per);
        const bool in = gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2;
        for (int k = 0; k < 25; ++k)
          out[base + (size_t)(col * 25 + k) * pp + e] = in ? tabs[l][((size_t)gy * nq + gx) * 50 + half * 25 + k] : 0.0;
      }
    base += (size_t)225 * pp;
  }
}

// The Q1 counterpart for the pressure hierarchies (no convection): levels
// n0 <= kQ1SmallN .. 2 of the unconstrained grids in one work-group per grid.
// A 32-node tile covers them, so the tiled smoother is plain four-colour
// Gauss-Seidel (colour 2 (gy % 2) + gx % 2); residual, restriction (1/2, 1,
// 1/2), the coarsest solve with node 0 held at zero (FP64 accumulation, as in
// k_q1_coarse_solve) and prolongation follow the per-level kernels.
namespace {
constexpr int kQ1SmallEntries = sq(kQ1SmallN + 1) + sq(kQ1SmallN / 2 + 1) + sq(kQ1SmallN / 4 + 1) + sq(kQ1SmallN / 8 + 1);

// (A x)(gx, gy) and the diagonal of alpha M + gamma K on the unconstrained grid
template <typename R>
__device__ __forceinline__ void q1_small_apply(const cpx<R>* x, int n, int gx, int gy, double h, const OpR<R>& o,
                                               cpx<R>& ax, cpx<R>& dg) {
  const int np = n + 1;
  R mx[3], kx[3], my[3], ky[3];
  q1_rows_r<R>(gx, n, h, mx, kx);
  q1_rows_r<R>(gy, n, h, my, ky);
  R amr = 0, ami = 0, akr = 0, aki = 0;
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
    const int jy = gy + dy - 1;
    if (jy < 0 || jy > n) continue;
    R smr = 0, smi = 0, skr = 0, ski = 0;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int jx = gx + dx - 1;
      if (jx < 0 || jx > n) continue;
      const cpx<R> v = x[jy * np + jx];
      smr += mx[dx] * v.x; smi += mx[dx] * v.y;
      skr += kx[dx] * v.x; ski += kx[dx] * v.y;
    }
    amr += my[dy] * smr; ami += my[dy] * smi;
    akr += ky[dy] * smr + my[dy] * skr; aki += ky[dy] * smi + my[dy] * ski;
  }
  ax.x = o.ar * amr - o.ai * ami + o.gr * akr - o.gi * aki;
  ax.y = o.ar * ami + o.ai * amr + o.gr * aki + o.gi * akr;
  const R md = mx[1] * my[1], kd = kx[1] * my[1] + mx[1] * ky[1];
  dg.x = o.ar * md + o.gr * kd;
  dg.y = o.ai * md + o.gi * kd;
}

template <typename R>
__device__ __forceinline__ void q1_small_sweep(cpx<R>* x, const cpx<R>* b, int n, const OpR<R>& o, bool forward) {
  const int np = n + 1, half = (np + 1) / 2;
  const double h = 1.0 / n;
  for (int k = 0; k < 4; ++k) {
    const int col = forward ? k : 3 - k;
    for (int e = threadIdx.x; e < half * half; e += blockDim.x) {
      const int gx = col % 2 + 2 * (e % half), gy = col / 2 + 2 * (e / half);
      if (gx > n || gy > n) continue;
      cpx<R> ax, dg;
      q1_small_apply<R>(x, n, gx, gy, h, o, ax, dg);
      const cpx<R> bv = b[gy * np + gx];
      const R er = bv.x - ax.x, ei = bv.y - ax.y;
      const R den = dg.x * dg.x + dg.y * dg.y;
      cpx<R>& xs = x[gy * np + gx];
      cpx<R> nv;
      nv.x = xs.x + (er * dg.x + ei * dg.y) / den;
      nv.y = xs.y + (ei * dg.x - er * dg.y) / den;
      xs = nv;
    }
    __syncthreads();
  }
}
}  // namespace

template <typename R>
__global__ __launch_bounds__(256) void k_q1_small_vcycle(cpx<R>* xg, const cpx<R>* x0, const cpx<R>* __restrict__ bg,
                                                         int n0, const OpCoef* __restrict__ coef, int fpc,
                                                         const double2* __restrict__ inv, int nb, Mask mk) {
  __shared__ cpx<R> xs[kQ1SmallEntries], bs[kQ1SmallEntries], rs[sq(kQ1SmallN + 1)];
  const int f = blockIdx.x;
  if (f >= nb || mk.off(f)) return;
  const OpR<R> o(coef[f / fpc]);
  int lev = 0, off[8], nn[8];
  for (int n = n0, q = 0; n >= 2; n >>= 1, ++lev) { off[lev] = q; nn[lev] = n; q += sq(n + 1); }
  const int np0 = n0 + 1;
  const size_t g0 = (size_t)f * np0 * np0;
  for (int e = threadIdx.x; e < np0 * np0; e += blockDim.x) {
    bs[e] = bg[g0 + e];
    xs[e] = x0 ? x0[g0 + e] : cmk<cpx<R>>(0, 0);
  }
  for (int e = np0 * np0 + threadIdx.x; e < off[lev - 1] + 9; e += blockDim.x) xs[e] = cmk<cpx<R>>(0, 0);
  __syncthreads();
  for (int l = 0; l + 1 < lev; ++l) {
    const int n = nn[l], np = n + 1, nc = n / 2, npc = nc + 1;
    cpx<R>* x = xs + off[l];
    const cpx<R>* b = bs + off[l];
    q1_small_sweep<R>(x, b, n, o, true);
    const double h = 1.0 / n;
    for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
      cpx<R> ax, dg;
      q1_small_apply<R>(x, n, e % np, e / np, h, o, ax, dg);
      cpx<R> r;
      r.x = b[e].x - ax.x;
      r.y = b[e].y - ax.y;
      rs[e] = r;
    }
    __syncthreads();
    cpx<R>* bc = bs + off[l + 1];
    const R w[3] = {R(0.5), R(1), R(0.5)};
    for (int e = threadIdx.x; e < npc * npc; e += blockDim.x) {
      const int I = e % npc, J = e / npc;
      cpx<R> v = cmk<cpx<R>>(0, 0);
      for (int dy = 0; dy < 3; ++dy) {
        const int fy = 2 * J + dy - 1;
        if (fy < 0 || fy > n) continue;
        for (int dx = 0; dx < 3; ++dx) {
          const int fx = 2 * I + dx - 1;
          if (fx < 0 || fx > n) continue;
          const cpx<R> rv = rs[fy * np + fx];
          v.x += w[dx] * w[dy] * rv.x;
          v.y += w[dx] * w[dy] * rv.y;
        }
      }
      bc[e] = v;
    }
    __syncthreads();
  }
  {   // coarsest grid (N = 2): node 0 held at zero, 8 x 8 inverse for nodes 1..8
    const cpx<R>* b = bs + off[lev - 1];
    cpx<R>* x = xs + off[lev - 1];
    const double2* A = inv + (size_t)(f / fpc) * 64;
    if (threadIdx.x < 9) {
      const int r = threadIdx.x;
      double sr = 0, si = 0;
      if (r > 0) {
        for (int q = 0; q < 8; ++q) {
          const cpx<R> v = b[1 + q];
          const double2 a = A[(r - 1) * 8 + q];
          sr += a.x * (double)v.x - a.y * (double)v.y;
          si += a.x * (double)v.y + a.y * (double)v.x;
        }
      }
      x[r] = cmk<cpx<R>>(sr, si);
    }
    __syncthreads();
  }
  for (int l = lev - 2; l >= 0; --l) {
    const int n = nn[l], np = n + 1, npc = n / 2 + 1;
    cpx<R>* x = xs + off[l];
    const cpx<R>* ec = xs + off[l + 1];
    for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
      const cpx<R> p = q1_prolong_at<R>(ec, npc, e % np, e / np);
      x[e].x += p.x;
      x[e].y += p.y;
    }
    __syncthreads();
    q1_small_sweep<R>(x, bs + off[l], n, o, false);
  }
  for (int e = threadIdx.x; e < np0 * np0; e += blockDim.x) xg[g0 + e] = xs[e];
}

template <typename R>
void launch_q1_small_vcycle(hipStream_t s, cpx<R>* x, const cpx<R>* x0, const cpx<R>* b, int n0, const OpCoef* coef,
                            int fpc, const double2* inv, int nb, Mask mk) {
  hipLaunchKernelGGL(k_q1_small_vcycle<R>, dim3((unsigned)nb), dim3(256), 0, s, x, x0, b, n0, coef, fpc, inv, nb, mk);
}

// ---------------------------------------------------------------- Chebyshev
// One step of the Jacobi-preconditioned Chebyshev semi-iteration for the
// mass matrix (Q2 interior or Q1 unconstrained):
//   first:  xn = g D^{-1} b
//   else:   xn = w (x - xp + g D^{-1}(b - M x)) + xp
// xn may alias xp (each thread reads its own xp entry before writing);
// xp == nullptr stands for x_{k-1} = 0 (the second step).
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
  const R gr = (R)g, wr = (R)w;
  if (first) {
    R mx[5], kx[5], my[5], ky[5];
    q2_rows_r<R>(ix, h, mx, kx); q2_rows_r<R>(iy, h, my, ky);
    const R d = mx[2] * my[2];
    const cpx<R> bi = b[i];
    cpx<R> v;
    v.x = gr * bi.x / d;
    v.y = gr * bi.y / d;
    xn[i] = v;
    return;
  }
  cpx<R> ax, dg;
  q2_apply_node<R>(x + (size_t)f * nq * nq, nq, ix, iy, h, c, nullptr, ax, dg);
  const cpx<R> bi = b[i], xi = x[i], pi = xp ? xp[i] : cmk<cpx<R>>(0, 0);
  const R d = dg.x;
  cpx<R> v;
  v.x = wr * (xi.x - pi.x + gr * (bi.x - ax.x) / d) + pi.x;
  v.y = wr * (xi.y - pi.y + gr * (bi.y - ax.y) / d) + pi.y;
  xn[i] = v;
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
  const R gr = (R)g, wr = (R)w;
  if (first) {
    R mx[3], kx[3], my[3], ky[3];
    q1_rows_r<R>(ix, n, h, mx, kx); q1_rows_r<R>(iy, n, h, my, ky);
    const R d = mx[1] * my[1];
    const cpx<R> bi = b[i];
    cpx<R> v;
    v.x = gr * bi.x / d;
    v.y = gr * bi.y / d;
    xn[i] = v;
    return;
  }
  q1_apply_node<R>(x + (size_t)f * np * np, n, ix, iy, h, c, nullptr, ax, dg);
  const cpx<R> bi = b[i], xi = x[i], pi = xp ? xp[i] : cmk<cpx<R>>(0, 0);
  const R d = dg.x;
  cpx<R> v;
  v.x = wr * (xi.x - pi.x + gr * (bi.x - ax.x) / d) + pi.x;
  v.y = wr * (xi.y - pi.y + gr * (bi.y - ax.y) / d) + pi.y;
  xn[i] = v;
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

// ---------------------------------------------- global multicolour sweeps
// Gauss-Seidel (SOR with relaxation factor 1) over whole grids in the
// multicolour order, the smoother of section 3.4 as read for this method:
// one launch per colour, in place (nodes of one colour do not couple).  Q2
// colour (ix mod 3, iy mod 3) over the interior padded indices 1..2n-1, Q1
// colour (ix mod 2, iy mod 2) over all nodes 0..n.  ``conv``: per-node
// stencil table of the level (25 values of N, 25 of N^T per Q2 node), with
// coef.eta scaling N and coef.etat scaling N^T, or null.
template <typename R>
__global__ __launch_bounds__(256) void k_q2_colour(cpx<R>* x, const cpx<R>* __restrict__ b, int n, double h,
                                                   const OpCoef* __restrict__ coef, int fpc,
                                                   const double* __restrict__ conv, int cx, int cy, int mx, int my,
                                                   Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mx * my) return;
  const int nq = 2 * n + 1;
  const int ix = (cx == 0 ? 3 : cx) + 3 * (t % mx), iy = (cy == 0 ? 3 : cy) + 3 * (t / mx);
  cpx<R>* xf = x + (size_t)f * nq * nq;
  cpx<R> ax, dg;
  q2_apply_node<R>(xf, nq, ix, iy, h, coef[f / fpc], conv, ax, dg);
  const size_t i = (size_t)iy * nq + ix;
  const cpx<R> r = b[(size_t)f * nq * nq + i] - ax;
  const cpx<R> d = cdiv(r, dg);
  xf[i] = xf[i] + d;
}

template <typename R>
__global__ __launch_bounds__(256) void k_q1_colour(cpx<R>* x, const cpx<R>* __restrict__ b, int n, double h,
                                                   const OpCoef* __restrict__ coef, int fpc, int cx, int cy, int mx,
                                                   int my, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mx * my) return;
  const int np = n + 1;
  const int ix = cx + 2 * (t % mx), iy = cy + 2 * (t / mx);
  cpx<R>* xf = x + (size_t)f * np * np;
  cpx<R> ax, dg;
  q1_apply_node<R>(xf, n, ix, iy, h, coef[f / fpc], nullptr, ax, dg);
  const size_t i = (size_t)iy * np + ix;
  const cpx<R> r = b[(size_t)f * np * np + i] - ax;
  const cpx<R> d = cdiv(r, dg);
  xf[i] = xf[i] + d;
}

// 1-D Q2 interpolation from the coarse grid (coarse padded index c, fine i =
// 0..2 nf): a coarse vertex or midpoint coincides with fine nodes 4e and
// 4e + 2; the quarter points 4e + 1, 4e + 3 take the quadratic through the
// coarse element's three nodes at 1/4 and 3/4 of it.
__device__ __forceinline__ int q2_interp_1d(int i, int c[3], double w[3]) {
  const int e = i >> 2, r = i & 3;
  if (r == 0) { c[0] = 2 * e; w[0] = 1.0; return 1; }
  if (r == 2) { c[0] = 2 * e + 1; w[0] = 1.0; return 1; }
  c[0] = 2 * e; c[1] = 2 * e + 1; c[2] = 2 * e + 2;
  if (r == 1) { w[0] = 0.375; w[1] = 0.75; w[2] = -0.125; }
  else { w[0] = -0.125; w[1] = 0.75; w[2] = 0.375; }
  return 3;
}

// x = t + P ec on a Q2 level of n elements per side (coarse n / 2)
template <typename R>
__global__ __launch_bounds__(256) void k_q2_prolong_add(cpx<R>* __restrict__ x, const cpx<R>* __restrict__ t,
                                                        const cpx<R>* __restrict__ ec, int n, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int nq = 2 * n + 1, nqc = n + 1;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nq * nq) return;
  const int ix = k % nq, iy = k / nq;
  const size_t i = (size_t)f * nq * nq + k;
  if (ix == 0 || iy == 0 || ix == nq - 1 || iy == nq - 1) { x[i] = cmk<cpx<R>>(0, 0); return; }
  int cxs[3], cys[3];
  double wx[3], wy[3];
  const int nx = q2_interp_1d(ix, cxs, wx), ny = q2_interp_1d(iy, cys, wy);
  const cpx<R>* e = ec + (size_t)f * nqc * nqc;
  double sr = 0, si = 0;
  for (int a = 0; a < ny; ++a)
    for (int q = 0; q < nx; ++q) {
      const cpx<R> v = e[(size_t)cys[a] * nqc + cxs[q]];
      sr += wx[q] * wy[a] * (double)v.x;
      si += wx[q] * wy[a] * (double)v.y;
    }
  const cpx<R> tv = t[i];
  x[i] = cmk<cpx<R>>((double)tv.x + sr, (double)tv.y + si);
}

// x = t + P ec on a Q1 level (all nodes)
template <typename R>
__global__ __launch_bounds__(256) void k_q1_prolong_add(cpx<R>* __restrict__ x, const cpx<R>* __restrict__ t,
                                                        const cpx<R>* __restrict__ ec, int n, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int np = n + 1, npc = n / 2 + 1;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np * np) return;
  const size_t i = (size_t)f * np * np + k;
  const cpx<R> p = q1_prolong_at<R>(ec + (size_t)f * npc * npc, npc, k % np, k / np);
  x[i] = t[i] + p;
}

// ------------------------------------------------------------ launchers
static inline dim3 grid2(long work, int nb, int bs = 256) { return dim3((unsigned)((work + bs - 1) / bs), nb); }

template <typename R>
void launch_tile_sweep(hipStream_t s, bool q2, cpx<R>* xo, const cpx<R>* xi, const cpx<R>* b, const cpx<R>* ec,
                       int n, double h, const OpCoef* coef, int fpc, int nb, const void* conv, bool forward,
                       Mask mk) {
  if (q2) {
    launch_q2_sweep<R>(s, xo, xi, b, ec, n, h, coef, fpc, nb, (const R*)conv, forward, mk);
  } else {
    const int np = n + 1, ntx = (np + kT1 - 1) / kT1;
    hipLaunchKernelGGL(k_q1_tile_sweep<R>, dim3(ntx * ntx, nb), dim3(256), 0, s, xo, xi, b, ec, n, h, coef, fpc,
                       (const double*)conv, forward ? 1 : 0, ntx, mk);
  }
}

template <typename R>
void launch_colour_sweep(hipStream_t s, bool q2, cpx<R>* x, const cpx<R>* b, int n, double h, const OpCoef* coef,
                         int fpc, int nb, const double* conv, bool forward, Mask mk) {
  const int nc = q2 ? 9 : 4, m = q2 ? 3 : 2;
  for (int k = 0; k < nc; ++k) {
    const int c = forward ? k : nc - 1 - k;
    const int cx = c % m, cy = c / m;
    if (q2) {
      // interior padded indices 1..2n-1 with index mod 3 = c: first 3 (c = 0) or c
      auto cnt = [&](int c0) { const int f0 = c0 == 0 ? 3 : c0; return f0 > 2 * n - 1 ? 0 : (2 * n - 1 - f0) / 3 + 1; };
      const int mx = cnt(cx), my = cnt(cy);
      if (mx * my == 0) continue;
      hipLaunchKernelGGL(k_q2_colour<R>, grid2((long)mx * my, nb), dim3(256), 0, s, x, b, n, h, coef, fpc, conv, cx, cy,
                         mx, my, mk);
    } else {
      const int mx = (n - cx) / 2 + 1, my = (n - cy) / 2 + 1;
      hipLaunchKernelGGL(k_q1_colour<R>, grid2((long)mx * my, nb), dim3(256), 0, s, x, b, n, h, coef, fpc, cx, cy, mx,
                         my, mk);
    }
  }
}

template <typename R>
void launch_prolong_add(hipStream_t s, bool q2, cpx<R>* x, const cpx<R>* t, const cpx<R>* ec, int n, int nb,
                        Mask mk) {
  const long nn = q2 ? (long)(2 * n + 1) * (2 * n + 1) : (long)(n + 1) * (n + 1);
  if (q2) hipLaunchKernelGGL(k_q2_prolong_add<R>, grid2(nn, nb), dim3(256), 0, s, x, t, ec, n, mk);
  else hipLaunchKernelGGL(k_q1_prolong_add<R>, grid2(nn, nb), dim3(256), 0, s, x, t, ec, n, mk);
}

template <typename R>
void launch_q1_residual(hipStream_t s, cpx<R>* r, const cpx<R>* x, const cpx<R>* b, int n, double h,
                        const OpCoef* coef, int fpc, int nb, const double* conv, Mask mk) {
  const int np = n + 1;
  hipLaunchKernelGGL(k_q1_residual<R>, grid2((long)np * np, nb), dim3(256), 0, s, r, x, b, n, h, coef, fpc, conv, mk);
}

template <typename R>
void launch_apply(hipStream_t s, bool q2, cpx<R>* y, const cpx<R>* x, int n, double h, const OpCoef* coef,
                  int fpc, int nb, const void* conv, Mask mk) {
  if (q2) {
    launch_q2_apply<R>(s, y, x, nullptr, n, h, coef, fpc, nb, (const R*)conv, mk);
  } else {
    const int np = n + 1;
    hipLaunchKernelGGL(k_q1_apply<R>, grid2((long)np * np, nb), dim3(256), 0, s, y, x, n, h, coef, fpc,
                       (const double*)conv, mk);
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
    if (!first) return launch_q2_tile_cheb<R>(s, xn, x, xp, b, n, h, g, w, nb, mk);
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
  template void launch_colour_sweep<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, int, double, const OpCoef*, int,  \
                                       int, const double*, bool, Mask);                                              \
  template void launch_prolong_add<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, const cpx<R>*, int, int, Mask);    \
  template void launch_tile_sweep<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, int, \
                                     double, const OpCoef*, int, int, const void*, bool, Mask);                    \
  template void launch_q1_residual<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, int, double,          \
                                      const OpCoef*, int, int, const double*, Mask);                                 \
  template void launch_apply<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, int, double, const OpCoef*, int, int, \
                                const void*, Mask);                                                                \
  template void launch_q1_restrict<R>(hipStream_t, cpx<R>*, const cpx<R>*, int, int, Mask);                          \
  template void launch_coarse<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, const double2*, int, int, Mask);         \
  template void launch_cheb<R>(hipStream_t, bool, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, int,    \
                               double, double, double, int, int, Mask);                                              \
  template void launch_schur_combine_pin<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, const double2*, \
                                            int, int, int, Mask);                                                   \
  template void launch_q2_small_vcycle<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, int, const OpCoef*,  \
                                          int, int, const double2*, const R*, int, Mask);                            \
  template void launch_q1_small_vcycle<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, int, const OpCoef*,  \
                                          int, const double2*, int, Mask);

PINTOC_INST(double)
PINTOC_INST(float)

}  // namespace pintoc
