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
// m', k' that the compiler folds into the code.  Each wave serves one class at
// a time: the nodes with gx % 2 == PX, gy % 2 == PY of the current colour, 8 x 8
// of them per tile (one per 6 x 6 block), 3 entries apart inside a sub-grid.
//
// Colours and tiles are those of the tiled SOR: colour 3 (gy % 3) + gx % 3,
// tiles of 48 node indices aligned at node 0, Gauss-Seidel inside a tile and
// the values of the sweep's start for couplings to other tiles.
//
// Convection tables are reordered on the host per (tile, colour, class,
// stencil entry, lane), so the lanes of a wave read 64 consecutive doubles;
// every class slot holds 25 entries, so a sweep can load the next colour's
// entries of its lane (whatever its class) while the current colour computes.
//
// Lanes.  A class wave reads the nodes (la, lb) of the class's 8 x 8 nodes of
// the colour at sub-grid entries u = 3 la + 78 lb + const.  A 128-bit LDS read
// is served 16 lanes at a time; it runs without bank conflicts when every
// 16-lane group covers the 16 residues u mod 16 once and lane j of every group
// has the same residue (measured on gfx950).  Each residue occurs at exactly
// four nodes, so group g takes the g-th of them and lane 16 g + j the node of
// residue j.  Waves take the four classes in an order rotated per colour and
// per work-group, which spreads the heavy vertex-vertex class (25 points) over
// the SIMDs.
//
// Arithmetic runs in the storage precision R of the grids (FP64, or FP32 for
// the inner solves of the mixed-precision mode), so an FP32 sweep neither
// converts its operands nor holds FP64 registers.
//
// Work-group order is XCD-aware: ids are dealt round-robin to the 8 XCDs, so
// id g is remapped to v = (g % 8) (G / 8) + g / 8 and every XCD gets a
// contiguous range of v.  With a convection table v runs over grids fastest
// (a tile's table stays in one XCD's L2 while every grid of the batch uses it);
// without one it runs over tiles fastest (neighbouring tiles share halo lines).
#include "kernels.h"

namespace pintoc {

namespace {

constexpr int kT = 48;                 // tile side (node indices)
constexpr int kE = kT + 4;             // tile with halo
constexpr int kH = kE / 2;             // parity sub-grid side
constexpr int kSub = kH * kH + 4;      // sub-grid stride (entries; = 8 mod 16 for the row-order phases)
constexpr int kSP = kT;                // row pitch of the staged results of the operator tiles
// Staged results are row-major with one entry of skew per four rows.  The
// restriction gives the 16 lanes of a group a 4 x 4 block of coarse nodes, so
// they read fine entries 4 apart in x and 4 rows apart in y: with the pitch a
// multiple of 4 and the row skew the 16 entries fall on 16 different 16-byte
// residues (conflict-free 128-bit LDS reads).
__device__ __forceinline__ int stage_idx(int lx, int ly) { return ly * kSP + lx + (ly >> 2); }
static_assert((kT - 1) * kSP + (kT - 1) + (kT - 1) / 4 < 4 * kSub, "staged results fit the tile");

__host__ __device__ constexpr int wlen(int P) { return P ? 3 : 5; }
__host__ __device__ constexpr int wlo(int P) { return P ? -1 : -2; }
__host__ __device__ constexpr int cm0(int P) { return P ? 16 : 8; }    // centre of m'
__host__ __device__ constexpr int ck0(int P) { return P ? 16 : 14; }   // centre of k'
// Convection table block per (tile, colour): four class slots of kCE entries
// (a class uses wlen(PX) wlen(PY) of them), each entry 64 lanes wide.
constexpr int kCE = 25, kCC = 4 * kCE;
__host__ __device__ constexpr int coff(int PX, int PY) { return (PX + 2 * PY) * kCE; }
constexpr size_t kTileTab = (size_t)9 * kCC * 64;     // doubles per tile
// Tables are stored in the grids' precision R.  FP64 kernels load the next
// colour's entries into registers while the current colour computes; in FP32
// those registers cost more occupancy than the overlap gains, so the entries
// are read where used.
template <typename R> constexpr bool kTabPrefetch = sizeof(R) == 8;

// LDS offset of neighbour (dx, dy) from the base of a class-(PX, PY) node
template <int PX, int PY>
__device__ __forceinline__ constexpr int loff(int dx, int dy) {
  return (((PY + dy) & 1) * 2 + ((PX + dx) & 1)) * kSub + ((PY + 2 + dy) >> 1) * kH + ((PX + 2 + dx) >> 1);
}

// (m' . v, k' . v) along one direction for class P
template <int P> struct Comb;
template <> struct Comb<0> {
  template <typename T>
  static __device__ __forceinline__ void run(const T* v, T& m, T& k) {
    const T s04 = v[0] + v[4], s13 = v[1] + v[3];
    m = fma(T(8), v[2], fma(T(2), s13, -s04));
    k = fma(T(14), v[2], fma(T(-8), s13, s04));
  }
};
template <> struct Comb<1> {
  template <typename T>
  static __device__ __forceinline__ void run(const T* v, T& m, T& k) {
    const T s02 = v[0] + v[2];
    m = fma(T(16), v[1], T(2) * s02);
    k = fma(T(16), v[1], T(-8) * s02);
  }
};

// Lane (la, lb) of a class wave; see the comment at the top of the file.
__host__ __device__ __forceinline__ void lane_ab(int lane, int& la, int& lb) {
  const int g = lane >> 4, j = lane & 15;
  int cnt = 0;
  la = 0;
  lb = 0;
  for (int b = 0; b < 8; ++b) {
    const int a = (11 * (j - 14 * b + 256)) & 15;      // 3 a + 14 b = j (mod 16); 11 = 3^-1 mod 16
    if (a < 8) {
      if (cnt == g) { la = a; lb = b; }
      ++cnt;
    }
  }
}

// Tile-local coordinates of a lane's node of colour col in class (px, py).
__host__ __device__ __forceinline__ void node_of(int px, int py, int col, int la, int lb, int& lx, int& ly) {
  const int cx = col % 3, cy = col / 3;
  lx = cx + 3 * (2 * la + ((px - cx) & 1));
  ly = cy + 3 * (2 * lb + ((py - cy) & 1));
}

// class served by wave w at colour step k (0: (0,0), 1: (1,0), 2: (0,1), 3: (1,1))
__device__ __forceinline__ int class_of(int w, int k, int rot) { return (w + k + rot) & 3; }

// Uniform coefficients of a work-group in precision T: a = alpha h^2/900,
// g = gamma/90, e = eta.
template <typename T>
struct TCoef {
  T ar, ai, gr, gi, er, ei;
};

template <typename T>
__device__ __forceinline__ TCoef<T> tcoef(const OpCoef& c, double h) {
  const double s = h * h / 900.0;
  return TCoef<T>{(T)(c.alpha.x * s), (T)(c.alpha.y * s), (T)(c.gamma.x / 90.0), (T)(c.gamma.y / 90.0), (T)c.eta.x,
                  (T)c.eta.y};
}

// a Md + g Kd: diagonal without convection for class (PX, PY)
template <int PX, int PY, typename T>
__device__ __forceinline__ cpx<T> diag0(const TCoef<T>& t) {
  constexpr T md = cm0(PX) * cm0(PY), kd = ck0(PX) * cm0(PY) + cm0(PX) * ck0(PY);
  cpx<T> d;
  d.x = t.ar * md + t.gr * kd;
  d.y = t.ai * md + t.gi * kd;
  return d;
}

// Convection entries of a lane's node: held in registers (RegTab) or read
// where used from the tile table (GlobTab, stride 64 between entries).
template <typename R> struct RegTab {
  const R* t;
  __device__ __forceinline__ R operator()(int e) const { return t[e]; }
};
template <typename R> struct GlobTab {
  const R* p;
  __device__ __forceinline__ R operator()(int e) const { return p[e * 64]; }
};

// A x at a class-(PX, PY) node: base points at the node's sub-grid origin,
// tab gives its lane's convection entries.  Returns A x and the diagonal
// convection entry.
template <int PX, int PY, bool CV, typename R, typename Tab>
__device__ __forceinline__ cpx<R> stencil(const cpx<R>* base, const Tab& tab, const TCoef<R>& t, R& cdiag) {
  constexpr int nx = wlen(PX), ny = wlen(PY), lx0 = wlo(PX), ly0 = wlo(PY);
  R smr[ny], smi[ny], skr[ny], ski[ny];
  R cr = 0, ci = 0;
#pragma unroll
  for (int iy = 0; iy < ny; ++iy) {
    R vr[nx], vi[nx];
#pragma unroll
    for (int ix = 0; ix < nx; ++ix) {
      const cpx<R> v = base[loff<PX, PY>(lx0 + ix, ly0 + iy)];
      vr[ix] = v.x;
      vi[ix] = v.y;
      if (CV) {
        const R c = tab(iy * nx + ix);
        cr = fma(c, vr[ix], cr);
        ci = fma(c, vi[ix], ci);
      }
    }
    Comb<PX>::run(vr, smr[iy], skr[iy]);
    Comb<PX>::run(vi, smi[iy], ski[iy]);
  }
  R pmr, pmi, kmr, kmi, mkr, mki, unr, uni;
  Comb<PY>::run(smr, pmr, kmr);        // m'_y . (m'_x v),  k'_y . (m'_x v)
  Comb<PY>::run(smi, pmi, kmi);
  Comb<PY>::run(skr, mkr, unr);        // m'_y . (k'_x v)
  Comb<PY>::run(ski, mki, uni);
  const R pkr = mkr + kmr, pki = mki + kmi;
  cpx<R> ax;
  ax.x = t.ar * pmr - t.ai * pmi + t.gr * pkr - t.gi * pki;
  ax.y = t.ar * pmi + t.ai * pmr + t.gr * pki + t.gi * pkr;
  if (CV) {
    ax.x += t.er * cr - t.ei * ci;
    ax.y += t.er * ci + t.ei * cr;
    cdiag = tab((wlen(PY) / 2) * nx + nx / 2);
  }
  return ax;
}

// Load the convection entries of a lane's node at colour col into registers:
// class cls (wave-uniform) of the tile's table ctile.  Entry e is loaded only
// when the class uses it (a wave-uniform predicate), so the array stays
// statically indexed without reading a slot's unused entries.
template <typename R>
__device__ __forceinline__ void load_tab(R* tab, const R* __restrict__ ctile, int col, int cls, int lane) {
  const R* src = ctile + ((size_t)col * kCC + cls * kCE) * 64 + lane;
  const int ne = wlen(cls & 1) * wlen(cls >> 1);
#pragma unroll
  for (int e = 0; e < kCE; ++e)
    if (e < ne) tab[e] = src[e * 64];
}

__device__ __forceinline__ bool tile_of_block(int ntiles, int nb, bool grid_fast, int& tile, int& f) {
  const unsigned per = gridDim.x >> 3;
  const unsigned v = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  if (v >= (unsigned)ntiles * (unsigned)nb) return false;
  if (grid_fast) { tile = (int)(v / nb); f = (int)(v % nb); }
  else { f = (int)(v / ntiles); tile = (int)(v % ntiles); }
  return true;
}

__device__ __forceinline__ int sub_index(int ex, int ey) {
  return ((ey & 1) * 2 + (ex & 1)) * kSub + (ey >> 1) * kH + (ex >> 1);
}

// Load the tile and halo of x (zero when xi is null) into the parity
// sub-grids; boundary and outside nodes are zero.  Thread t < 4 kE owns column
// ex = t % kE and rows ey = t / kE + 4 k, so addresses advance by constant
// strides (coalesced along each row).
constexpr int kLR = kE / 4;            // rows per loading thread
static_assert(kE % 4 == 0 && 4 * kE <= 256, "tile loading layout");

template <typename R>
__device__ __forceinline__ void load_tile(cpx<R>* sx, const cpx<R>* __restrict__ xi, int nq, int X0, int Y0) {
  if (threadIdx.x >= 4 * kE) return;
  const int ex = (int)threadIdx.x % kE, ey0 = (int)threadIdx.x / kE;
  const int gx = X0 - 2 + ex, gy0 = Y0 - 2 + ey0;
  const bool xin = xi && gx >= 1 && gx <= nq - 2;
  const cpx<R>* src = xin ? xi + ((ptrdiff_t)gy0 * nq + gx) : xi;    // dereferenced only for nodes inside
  cpx<R> v[kLR];
#pragma unroll
  for (int k = 0; k < kLR; ++k) {
    const int gy = gy0 + 4 * k;
    v[k] = (xin && gy >= 1 && gy <= nq - 2) ? src[(ptrdiff_t)4 * k * nq] : cmk<cpx<R>>(0, 0);
  }
  cpx<R>* dst = sx + ((ey0 & 1) * 2 + (ex & 1)) * kSub + (ey0 >> 1) * kH + (ex >> 1);
#pragma unroll
  for (int k = 0; k < kLR; ++k) dst[2 * k * kH] = v[k];
}

// 1-D Q2 prolongation: fine node 4e + r from coarse nodes 2e, 2e + 1, 2e + 2.
template <typename T>
__device__ __forceinline__ void prolong_row(const T c[3], T f[4]) {
  f[0] = c[0];
  f[1] = T(0.375) * c[0] + T(0.75) * c[1] - T(0.125) * c[2];
  f[2] = c[1];
  f[3] = T(-0.125) * c[0] + T(0.75) * c[1] + T(0.375) * c[2];
}

// Load t + P ec (t: fine iterate, ec: coarse correction on the padded grid of
// side (nq + 1) / 2) for the tile and halo.  A thread builds one 4 x 4 block of
// fine nodes aligned with a coarse cell (fine 4e .. 4e + 3 per direction,
// coarse 2e .. 2e + 2) from 3 x 3 coarse values; 14 x 14 blocks cover
// [X0 - 4, X0 + 52).
constexpr int kPB = kE / 4 + 1;

template <typename R>
__device__ __forceinline__ void load_tile_prolong(cpx<R>* sx, const cpx<R>* __restrict__ xi,
                                                  const cpx<R>* __restrict__ ec, int nq, int X0, int Y0) {
  if (threadIdx.x >= kPB * kPB) return;
  const int nqc = (nq + 1) / 2;
  const int ex0 = X0 / 4 - 1 + (int)threadIdx.x % kPB, ey0 = Y0 / 4 - 1 + (int)threadIdx.x / kPB;
  cpx<R> c[9], tv[16];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int cx = 2 * ex0 + q, cy = 2 * ey0 + a;
      c[3 * a + q] = (cx >= 0 && cx < nqc && cy >= 0 && cy < nqc) ? ec[(size_t)cy * nqc + cx] : cmk<cpx<R>>(0, 0);
    }
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gx = 4 * ex0 + r, gy = 4 * ey0 + s2;
      const int ex = gx - X0 + 2, ey = gy - Y0 + 2;
      const bool load = xi && ex >= 0 && ex < kE && ey >= 0 && ey < kE && gx >= 1 && gx <= nq - 2 && gy >= 1 &&
                        gy <= nq - 2;
      tv[4 * s2 + r] = load ? xi[(size_t)gy * nq + gx] : cmk<cpx<R>>(0, 0);
    }
  R pr[3][4], pi[3][4];                // prolonged along x, per coarse row
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R cr[3] = {c[3 * a].x, c[3 * a + 1].x, c[3 * a + 2].x};
    const R ci[3] = {c[3 * a].y, c[3 * a + 1].y, c[3 * a + 2].y};
    prolong_row<R>(cr, pr[a]);
    prolong_row<R>(ci, pi[a]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const R colr[3] = {pr[0][r], pr[1][r], pr[2][r]}, coli[3] = {pi[0][r], pi[1][r], pi[2][r]};
    R fr[4], fi[4];
    prolong_row<R>(colr, fr);
    prolong_row<R>(coli, fi);
    const int gx = 4 * ex0 + r, ex = gx - X0 + 2;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int gy = 4 * ey0 + s2, ey = gy - Y0 + 2;
      if (ex < 0 || ex >= kE || ey < 0 || ey >= kE) continue;
      const bool in = gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2;
      const cpx<R> t = tv[4 * s2 + r];
      cpx<R> v;
      v.x = in ? t.x + fr[s2] : R(0);
      v.y = in ? t.y + fi[s2] : R(0);
      sx[sub_index(ex, ey)] = v;
    }
  }
}

// b at the lane's node of every colour step k (class and colour of that step).
template <typename R, bool FWD>
__device__ __forceinline__ void prefetch_b(cpx<R>* bb, const cpx<R>* __restrict__ bf, int w, int rot, int la, int lb,
                                           int X0, int Y0, int nq) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int col = FWD ? k : 8 - k, c = class_of(w, k, rot);
    int lx, ly;
    node_of(c & 1, c >> 1, col, la, lb, lx, ly);
    const int gx = X0 + lx, gy = Y0 + ly;
    bb[k] = (gx >= 1 && gx <= nq - 2 && gy >= 1 && gy <= nq - 2) ? bf[(size_t)gy * nq + gx] : cmk<cpx<R>>(0, 0);
  }
}

// One colour of the sweep for a lane of class (PX, PY).  dinv: inverse of the
// class diagonal (used without convection, where it is uniform).
template <int PX, int PY, bool CV, typename R>
__device__ __forceinline__ void sweep_node(cpx<R>* sx, int col, int la, int lb, int lane, int X0, int Y0, int nq,
                                           cpx<R> bv, const TCoef<R>& t, cpx<R> dinv, const R* tab,
                                           const R* __restrict__ ctile) {
  int lx, ly;
  node_of(PX, PY, col, la, lb, lx, ly);
  const int gx = X0 + lx, gy = Y0 + ly;
  if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) return;
  cpx<R>* base = sx + ((ly - PY) >> 1) * kH + ((lx - PX) >> 1);
  R cd = 0;
  cpx<R> ax;
  if (kTabPrefetch<R>)
    ax = stencil<PX, PY, CV, R>(base, RegTab<R>{tab}, t, cd);
  else
    ax = stencil<PX, PY, CV, R>(base, GlobTab<R>{CV ? ctile + ((size_t)col * kCC + coff(PX, PY)) * 64 + lane : nullptr},
                                t, cd);
  if (CV) {
    cpx<R> d = diag0<PX, PY, R>(t);
    d.x += t.er * cd;
    d.y += t.ei * cd;
    const R inv = R(1) / (d.x * d.x + d.y * d.y);
    dinv.x = d.x * inv;
    dinv.y = -d.y * inv;
  }
  const R er = bv.x - ax.x, ei = bv.y - ax.y;
  cpx<R>& xs = base[loff<PX, PY>(0, 0)];
  cpx<R> nx;
  nx.x = xs.x + er * dinv.x - ei * dinv.y;
  nx.y = xs.y + er * dinv.y + ei * dinv.x;
  xs = nx;
}

template <int PX, int PY, typename R>
__device__ __forceinline__ cpx<R> inv_diag0(const TCoef<R>& t) {
  const cpx<R> d = diag0<PX, PY, R>(t);
  const R inv = R(1) / (d.x * d.x + d.y * d.y);
  cpx<R> v;
  v.x = d.x * inv;
  v.y = -d.y * inv;
  return v;
}

// Write the tile interior from LDS (or zero on boundary nodes) to xo.  Thread
// t < 5 kT owns column lx = t % kT and rows ly = t / kT + 5 k.
constexpr int kSR = (kT + 4) / 5;      // rows per storing thread (the last may fall outside)
static_assert(5 * kT <= 256, "tile storing layout");

template <typename R>
__device__ __forceinline__ void store_tile(cpx<R>* __restrict__ xo, const cpx<R>* sx, int nq, int X0, int Y0) {
  if (threadIdx.x >= 5 * kT) return;
  const int lx = (int)threadIdx.x % kT, ly0 = (int)threadIdx.x / kT;
  const int gx = X0 + lx;
  if (gx >= nq) return;
  const bool xin = gx >= 1 && gx <= nq - 2;
  cpx<R>* dst = xo + (ptrdiff_t)(Y0 + ly0) * nq + gx;
#pragma unroll
  for (int k = 0; k < kSR; ++k) {
    const int ly = ly0 + 5 * k, gy = Y0 + ly;
    if (ly >= kT || gy >= nq) break;
    const bool in = xin && gy >= 1 && gy <= nq - 2;
    dst[(ptrdiff_t)5 * k * nq] = in ? sx[sub_index(lx + 2, ly + 2)] : cmk<cpx<R>>(0, 0);
  }
}

}  // namespace

// Sweep x -> xo.  xi == nullptr: start from x = 0.  PRO: start from xi + P ec
// (the coarse-grid correction of the V-cycle, applied while loading).
template <typename R, bool CV, bool FWD, bool PRO>
__global__ __launch_bounds__(256) void k_q2_sweep(cpx<R>* __restrict__ xo, const cpx<R>* __restrict__ xi,
                                                  const cpx<R>* __restrict__ b, const cpx<R>* __restrict__ ec, int n,
                                                  double h, const OpCoef* __restrict__ coef, int fpc,
                                                  const R* __restrict__ conv, int ntx, int nb, Mask mk) {
  __shared__ cpx<R> sx[4 * kSub];
  int tile, f;
  if (!tile_of_block(ntx * ntx, nb, CV, tile, f)) return;
  if (mk.off(f)) return;
  const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
  const int nq = 2 * n + 1, nqc = n + 1;
  const size_t off = (size_t)f * nq * nq;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, rot = (int)(blockIdx.x >> 3) & 3;
  int la, lb;
  lane_ab(lane, la, lb);
  cpx<R> bb[9];
  prefetch_b<R, FWD>(bb, b + off, w, rot, la, lb, X0, Y0, nq);
  if (PRO) load_tile_prolong<R>(sx, xi ? xi + off : nullptr, ec + (size_t)f * nqc * nqc, nq, X0, Y0);
  else load_tile<R>(sx, xi ? xi + off : nullptr, nq, X0, Y0);
  const TCoef<R> t = tcoef<R>(coef[f / fpc], h);
  cpx<R> dv0 = cmk<cpx<R>>(0, 0), dv1 = dv0, dv2 = dv0, dv3 = dv0;
  if (!CV) {
    dv0 = inv_diag0<0, 0, R>(t);
    dv1 = inv_diag0<1, 0, R>(t);
    dv2 = inv_diag0<0, 1, R>(t);
    dv3 = inv_diag0<1, 1, R>(t);
  }
  // Convection entries: those of colour step k + 1 are loaded while step k
  // computes, so their latency overlaps the step.
  const R* ctile = CV ? conv + (size_t)tile * kTileTab : nullptr;
  constexpr bool PF = CV && kTabPrefetch<R>;
  R tcur[PF ? kCE : 1], tnxt[PF ? kCE : 1];
  if (PF) load_tab<R>(tcur, ctile, FWD ? 0 : 8, class_of(w, 0, rot), lane);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int col = FWD ? k : 8 - k;
    if (PF && k < 8) load_tab<R>(tnxt, ctile, FWD ? k + 1 : 7 - k, class_of(w, k + 1, rot), lane);
    switch (class_of(w, k, rot)) {
      case 0: sweep_node<0, 0, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, bb[k], t, dv0, tcur, ctile); break;
      case 1: sweep_node<1, 0, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, bb[k], t, dv1, tcur, ctile); break;
      case 2: sweep_node<0, 1, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, bb[k], t, dv2, tcur, ctile); break;
      default: sweep_node<1, 1, CV, R>(sx, col, la, lb, lane, X0, Y0, nq, bb[k], t, dv3, tcur, ctile); break;
    }
    __syncthreads();
    if (PF) {
#pragma unroll
      for (int e = 0; e < kCE; ++e) tcur[e] = tnxt[e];
    }
  }
  store_tile<R>(xo + off, sx, nq, X0, Y0);
}

namespace {
template <int PX, int PY, bool CV, typename R>
__device__ __forceinline__ cpx<R> apply_node(const cpx<R>* sx, int col, int la, int lb, int lane, int X0, int Y0,
                                             int nq, const TCoef<R>& t, const R* tab,
                                             const R* __restrict__ ctile, int& si) {
  int lx, ly;
  node_of(PX, PY, col, la, lb, lx, ly);
  si = stage_idx(lx, ly);
  const int gx = X0 + lx, gy = Y0 + ly;
  if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) return cmk<cpx<R>>(0, 0);
  const cpx<R>* base = sx + ((ly - PY) >> 1) * kH + ((lx - PX) >> 1);
  R cd = 0;
  if (kTabPrefetch<R>) return stencil<PX, PY, CV, R>(base, RegTab<R>{tab}, t, cd);
  return stencil<PX, PY, CV, R>(base, GlobTab<R>{CV ? ctile + ((size_t)col * kCC + coff(PX, PY)) * 64 + lane : nullptr},
                                t, cd);
}

// Load x into the tile and leave A x of every tile node staged row-major
// (stage_idx layout) in the LDS tile (zero on boundary and outside nodes).
template <typename R, bool CV>
__device__ __forceinline__ void apply_stage(cpx<R>* sx, const cpx<R>* __restrict__ x, int nq, int X0, int Y0,
                                            const TCoef<R>& t, const R* __restrict__ ctile, int w, int lane,
                                            int rot) {
  int la, lb;
  lane_ab(lane, la, lb);
  constexpr bool PF = CV && kTabPrefetch<R>;
  R tcur[PF ? kCE : 1], tnxt[PF ? kCE : 1];
  if (PF) load_tab<R>(tcur, ctile, 0, class_of(w, 0, rot), lane);
  load_tile<R>(sx, x, nq, X0, Y0);
  __syncthreads();
  cpx<R> acc[9];
  int si[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (PF && k < 8) load_tab<R>(tnxt, ctile, k + 1, class_of(w, k + 1, rot), lane);
    switch (class_of(w, k, rot)) {
      case 0: acc[k] = apply_node<0, 0, CV, R>(sx, k, la, lb, lane, X0, Y0, nq, t, tcur, ctile, si[k]); break;
      case 1: acc[k] = apply_node<1, 0, CV, R>(sx, k, la, lb, lane, X0, Y0, nq, t, tcur, ctile, si[k]); break;
      case 2: acc[k] = apply_node<0, 1, CV, R>(sx, k, la, lb, lane, X0, Y0, nq, t, tcur, ctile, si[k]); break;
      default: acc[k] = apply_node<1, 1, CV, R>(sx, k, la, lb, lane, X0, Y0, nq, t, tcur, ctile, si[k]); break;
    }
    if (PF) {
#pragma unroll
      for (int e = 0; e < kCE; ++e) tcur[e] = tnxt[e];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 9; ++k) sx[si[k]] = acc[k];
  __syncthreads();
}
}  // namespace

// out = b - A x (b != nullptr) or out = A x, on every node of the grids
// (zero on the boundary).  out and x must not alias.
template <typename R, bool CV>
__global__ __launch_bounds__(256) void k_q2_tile_apply(cpx<R>* __restrict__ out, const cpx<R>* __restrict__ x,
                                                       const cpx<R>* __restrict__ b, int n, double h,
                                                       const OpCoef* __restrict__ coef, int fpc,
                                                       const R* __restrict__ conv, int ntx, int nb, Mask mk) {
  __shared__ cpx<R> sx[4 * kSub];
  int tile, f;
  if (!tile_of_block(ntx * ntx, nb, CV, tile, f)) return;
  if (mk.off(f)) return;
  const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
  const int nq = 2 * n + 1;
  const size_t off = (size_t)f * nq * nq;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, rot = (int)(blockIdx.x >> 3) & 3;
  const TCoef<R> t = tcoef<R>(coef[f / fpc], h);
  const R* ctile = CV ? conv + (size_t)tile * kTileTab : nullptr;
  apply_stage<R, CV>(sx, x + off, nq, X0, Y0, t, ctile, w, lane, rot);     // A x staged for a coalesced store
  if (threadIdx.x < 5 * kT) {
    const int lx = (int)threadIdx.x % kT, ly0 = (int)threadIdx.x / kT;
    const int gx = X0 + lx;
    if (gx < nq) {
      const bool xin = gx >= 1 && gx <= nq - 2;
      const ptrdiff_t g0 = (ptrdiff_t)off + (ptrdiff_t)(Y0 + ly0) * nq + gx;
#pragma unroll
      for (int k = 0; k < kSR; ++k) {
        const int ly = ly0 + 5 * k, gy = Y0 + ly;
        if (ly >= kT || gy >= nq) break;
        const ptrdiff_t g = g0 + (ptrdiff_t)5 * k * nq;
        const bool in = xin && gy >= 1 && gy <= nq - 2;
        cpx<R> v = in ? sx[stage_idx(lx, ly)] : cmk<cpx<R>>(0, 0);
        if (b) v = in ? b[g] - v : cmk<cpx<R>>(0, 0);
        out[g] = v;
      }
    }
  }
}

// Residual and restriction in one pass: bc = P^T (b - A x) on the coarse grid
// (side n + 1, zero on its boundary).  The fine tile of tile (tx, ty) reaches
// the coarse nodes 24 tx .. 24 tx + 24 per direction (1-D weights of an even
// coarse node at fine offsets -3, -1, 0, 1, 3: -1/8, 3/8, 1, 3/8, -1/8; of an
// odd one at -1, 0, 1: 3/4, 1, 3/4).  The work-group writes its own coarse
// nodes (local index < 24 in both directions) to bc and the partial sums of the
// shared column (local x index 24, 25 values) and row (local y index 24, 24
// values) to side[(f * ntiles + tile) * 49 + ...]; k_q2_restrict_fix adds those
// to the neighbours' nodes.  The fine residual never goes to memory.
namespace {
constexpr int kCT = kT / 2;            // coarse nodes owned per tile and direction
constexpr int kSide = 2 * kCT + 1;     // shared partial sums per tile: column (25) then row (24)

// 1-D restriction weight of fine offset index i (offsets -3, -1, 0, 1, 3) for coarse parity P
template <int P> __device__ __forceinline__ constexpr double rw(int i) {
  return P ? (i == 1 || i == 3 ? 0.75 : (i == 2 ? 1.0 : 0.0))
           : (i == 0 || i == 4 ? -0.125 : (i == 1 || i == 3 ? 0.375 : 1.0));
}
__device__ __forceinline__ constexpr int roff(int i) { return i == 0 ? -3 : (i == 4 ? 3 : i - 2); }

// Coarse nodes of parity class (PI, PJ) of the tile: local (2 a + PI, 2 b + PJ).
template <int PI, int PJ, typename R>
__device__ __forceinline__ void restrict_class(cpx<R>* __restrict__ bcf, cpx<R>* __restrict__ sd, const cpx<R>* sr,
                                               int I0, int J0, int nqc) {
  constexpr int na = PI ? kCT / 2 : kCT / 2 + 1, nbj = PJ ? kCT / 2 : kCT / 2 + 1;
  constexpr int nbx = (na + 3) / 4;
  static_assert(16 * nbx * ((nbj + 3) / 4) <= 256, "one coarse node per thread");
  // lane group g = threadIdx / 16 takes a 4 x 4 block of the class's coarse nodes
  {
    const int e = (int)threadIdx.x, g = e >> 4;
    const int ia = 4 * (g % nbx) + (e & 3), ib = 4 * (g / nbx) + ((e >> 2) & 3);
    if (ia >= na || ib >= nbj) return;
    const int ci = 2 * ia + PI, cj = 2 * ib + PJ;
    const int I = I0 + ci, J = J0 + cj;
    if (I >= nqc || J >= nqc) return;
    R vr = 0, vi = 0;
#pragma unroll
    for (int iy = 0; iy < 5; ++iy) {
      if (rw<PJ>(iy) == 0.0) continue;
      const int fy = 2 * cj + roff(iy);
      if (fy < 0 || fy >= kT) continue;
      R rr = 0, ri = 0;
#pragma unroll
      for (int ix = 0; ix < 5; ++ix) {
        if (rw<PI>(ix) == 0.0) continue;
        const int fx = 2 * ci + roff(ix);
        if (fx < 0 || fx >= kT) continue;
        const cpx<R> v = sr[stage_idx(fx, fy)];
        rr = fma((R)rw<PI>(ix), v.x, rr);
        ri = fma((R)rw<PI>(ix), v.y, ri);
      }
      vr = fma((R)rw<PJ>(iy), rr, vr);
      vi = fma((R)rw<PJ>(iy), ri, vi);
    }
    const bool bnd = I == 0 || J == 0 || I == nqc - 1 || J == nqc - 1;
    cpx<R> v;
    v.x = bnd ? R(0) : vr;
    v.y = bnd ? R(0) : vi;
    if (ci < kCT && cj < kCT) bcf[(size_t)J * nqc + I] = v;
    else if (ci == kCT) sd[cj] = v;
    else sd[kCT + 1 + ci] = v;
  }
}
}  // namespace

template <typename R, bool CV>
__global__ __launch_bounds__(256) void k_q2_residual_restrict(cpx<R>* __restrict__ bc, cpx<R>* __restrict__ side,
                                                              const cpx<R>* __restrict__ x,
                                                              const cpx<R>* __restrict__ b, int n, double h,
                                                              const OpCoef* __restrict__ coef, int fpc,
                                                              const R* __restrict__ conv, int ntx, int nb,
                                                              Mask mk) {
  __shared__ cpx<R> sx[4 * kSub];
  int tile, f;
  if (!tile_of_block(ntx * ntx, nb, CV, tile, f)) return;
  if (mk.off(f)) return;
  const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
  const int nq = 2 * n + 1, nqc = n + 1;
  const size_t off = (size_t)f * nq * nq;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, rot = (int)(blockIdx.x >> 3) & 3;
  const TCoef<R> t = tcoef<R>(coef[f / fpc], h);
  const R* ctile = CV ? conv + (size_t)tile * kTileTab : nullptr;
  // b of this thread's column rows (thread t < 5 kT: column t % kT, rows t / kT + 5 k);
  // in FP64 without convection it is loaded before the stencil phase so its
  // latency overlaps it (in FP32, or beside the convection table reads, the
  // registers cost more than the overlap gains)
  constexpr bool kPre = sizeof(R) == 8 && !CV;
  const int lx = (int)threadIdx.x % kT, ly0 = (int)threadIdx.x / kT;
  const int gx = X0 + lx;
  const bool xin = threadIdx.x < 5 * kT && gx >= 1 && gx <= nq - 2;
  const cpx<R>* bp = b + off + (ptrdiff_t)(Y0 + ly0) * nq + gx;
  auto bload = [&](int k) -> cpx<R> {
    const int gy = Y0 + ly0 + 5 * k;
    return (xin && ly0 + 5 * k < kT && gy >= 1 && gy <= nq - 2) ? bp[(ptrdiff_t)5 * k * nq] : cmk<cpx<R>>(0, 0);
  };
  cpx<R> bv[kSR];
  if constexpr (kPre) {
#pragma unroll
    for (int k = 0; k < kSR; ++k) bv[k] = bload(k);
  }
  apply_stage<R, CV>(sx, x + off, nq, X0, Y0, t, ctile, w, lane, rot);
  // r = b - A x in place over the staged A x (A x and b are zero on boundary and outside nodes)
  if (threadIdx.x < 5 * kT) {
#pragma unroll
    for (int k = 0; k < kSR; ++k) {
      const int ly = ly0 + 5 * k;
      if (ly >= kT) break;
      if constexpr (!kPre) bv[k] = bload(k);
      const cpx<R> a = sx[stage_idx(lx, ly)];
      cpx<R> r;
      r.x = bv[k].x - a.x;
      r.y = bv[k].y - a.y;
      sx[stage_idx(lx, ly)] = r;
    }
  }
  __syncthreads();
  cpx<R>* bcf = bc + (size_t)f * nqc * nqc;
  cpx<R>* sd = side + ((size_t)f * ntx * ntx + tile) * kSide;
  const int I0 = X0 / 2, J0 = Y0 / 2;
  restrict_class<0, 0, R>(bcf, sd, sx, I0, J0, nqc);
  restrict_class<1, 0, R>(bcf, sd, sx, I0, J0, nqc);
  restrict_class<0, 1, R>(bcf, sd, sx, I0, J0, nqc);
  restrict_class<1, 1, R>(bcf, sd, sx, I0, J0, nqc);
}

// One Chebyshev step for the Q2 mass matrix (not the first):
//   xn = w (x - xp + g D^{-1} (b - M x)) + xp      (D = diag(M), zero boundary)
// with M x formed on the LDS tile.  xn may alias xp (each node's xp is read
// by the thread that writes it); xp == nullptr stands for x_{k-1} = 0.
template <typename R>
__global__ __launch_bounds__(256) void k_q2_tile_cheb(cpx<R>* xn, const cpx<R>* __restrict__ x, const cpx<R>* xp,
                                                      const cpx<R>* __restrict__ b, int n, double h, double g,
                                                      double w, int ntx, int nb, Mask mk) {
  __shared__ cpx<R> sx[4 * kSub];
  int tile, f;
  if (!tile_of_block(ntx * ntx, nb, false, tile, f)) return;
  if (mk.off(f)) return;
  const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
  const int nq = 2 * n + 1;
  const size_t off = (size_t)f * nq * nq;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rot = (int)(blockIdx.x >> 3) & 3;
  const TCoef<R> t{(R)(h * h / 900.0), R(0), R(0), R(0), R(0), R(0)};
  apply_stage<R, false>(sx, x + off, nq, X0, Y0, t, nullptr, wv, lane, rot);      // M x staged row-major
  if (threadIdx.x >= 5 * kT) return;
  const int lx = (int)threadIdx.x % kT, ly0 = (int)threadIdx.x / kT, gx = X0 + lx;
  if (gx >= nq) return;
  const R gr = (R)g, wr = (R)w;
#pragma unroll
  for (int k = 0; k < kSR; ++k) {
    const int ly = ly0 + 5 * k, gy = Y0 + ly;
    if (ly >= kT || gy >= nq) break;
    const size_t i = off + (size_t)gy * nq + gx;
    if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) {
      xn[i] = cmk<cpx<R>>(0, 0);
      continue;
    }
    const R d = (R)(cm0(gx & 1) * cm0(gy & 1)) * t.ar;
    const cpx<R> mx = sx[stage_idx(lx, ly)], xi = x[i], pi = xp ? xp[i] : cmk<cpx<R>>(0, 0), bi = b[i];
    cpx<R> v;
    v.x = wr * (xi.x - pi.x + gr * (bi.x - mx.x) / d) + pi.x;
    v.y = wr * (xi.y - pi.y + gr * (bi.y - mx.y) / d) + pi.y;
    xn[i] = v;
  }
}

// Shared coarse nodes of k_q2_residual_restrict: I or J a positive multiple of
// 24 (interior nodes only).  Such a node adds the column partial of the tile
// to its left, the row partial of the tile below, and, when both I and J are
// multiples of 24, the corner partial of the tile below-left.  One thread per
// node, fixed summation order.
template <typename R>
__global__ __launch_bounds__(256) void k_q2_restrict_fix(cpx<R>* __restrict__ bc, const cpx<R>* __restrict__ side,
                                                         int n, int ntx, Mask mk) {
  const int f = blockIdx.y;
  if (mk.off(f)) return;
  const int nqc = n + 1, len = nqc - 2, A = len / kCT;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * A * len) return;
  const int line = e / len, pos = 1 + e % len;
  int I, J;
  if (line < A) {
    I = kCT * (line + 1);
    J = pos;
  } else {
    J = kCT * (line - A + 1);
    I = pos;
    if (I % kCT == 0) return;          // on a column line as well: done there
  }
  const int tx = I / kCT, ty = J / kCT, ci = I % kCT, cj = J % kCT;
  const cpx<R>* sd = side + (size_t)f * ntx * ntx * kSide;
  double vr = 0, vi = 0;
  if (ci == 0) {
    const cpx<R> v = sd[(size_t)(ty * ntx + tx - 1) * kSide + cj];
    vr += (double)v.x; vi += (double)v.y;
  }
  if (cj == 0) {
    const cpx<R> v = sd[(size_t)((ty - 1) * ntx + tx) * kSide + kCT + 1 + ci];
    vr += (double)v.x; vi += (double)v.y;
  }
  if (ci == 0 && cj == 0) {
    const cpx<R> v = sd[(size_t)((ty - 1) * ntx + tx - 1) * kSide + kCT];
    vr += (double)v.x; vi += (double)v.y;
  }
  cpx<R>& d = bc[(size_t)f * nqc * nqc + (size_t)J * nqc + I];
  d = cmk<cpx<R>>((double)d.x + vr, (double)d.y + vi);
}

namespace {
// Raw stencil sums at a class-(PX, PY) node: pm = m'.m' x, pk = (k'.m' + m'.k') x
// (so M x = h^2/900 pm, K x = pk/90) and the convection sum pc.
template <int PX, int PY, bool CV, typename R>
__device__ __forceinline__ void stencil_raw(const cpx<R>* base, const R* __restrict__ cn, cpx<R>& pm, cpx<R>& pk,
                                            cpx<R>& pc) {
  constexpr int nx = wlen(PX), ny = wlen(PY), lx0 = wlo(PX), ly0 = wlo(PY);
  R smr[ny], smi[ny], skr[ny], ski[ny];
  R cr = 0, ci = 0;
#pragma unroll
  for (int iy = 0; iy < ny; ++iy) {
    R vr[nx], vi[nx];
#pragma unroll
    for (int ix = 0; ix < nx; ++ix) {
      const cpx<R> v = base[loff<PX, PY>(lx0 + ix, ly0 + iy)];
      vr[ix] = v.x;
      vi[ix] = v.y;
      if (CV) {
        const R c = cn[(iy * nx + ix) * 64];
        cr = fma(c, vr[ix], cr);
        ci = fma(c, vi[ix], ci);
      }
    }
    Comb<PX>::run(vr, smr[iy], skr[iy]);
    Comb<PX>::run(vi, smi[iy], ski[iy]);
  }
  R pmr, pmi, kmr, kmi, mkr, mki, unr, uni;
  Comb<PY>::run(smr, pmr, kmr);
  Comb<PY>::run(smi, pmi, kmi);
  Comb<PY>::run(skr, mkr, unr);
  Comb<PY>::run(ski, mki, uni);
  pm.x = pmr; pm.y = pmi;
  pk.x = mkr + kmr; pk.y = mki + kmi;
  pc.x = cr; pc.y = ci;
}

template <typename R>
__device__ __forceinline__ cpx<R> cmad(cpx<R> acc, double2 cd, cpx<R> z) {     // acc + c z
  const R cx = (R)cd.x, cy = (R)cd.y;
  cpx<R> r;
  r.x = acc.x + cx * z.x - cy * z.y;
  r.y = acc.y + cx * z.y + cy * z.x;
  return r;
}

constexpr int kPP = kT / 2 + 2;       // side of the Q1 patch of a tile (26)

// Velocity rows of one frequency block (see oseen_kernels.hip for the block
// pattern) at a lane's node of colour col, phase 0 (v) or 1 (lambda):
//   phase 0: r1 = a11 M v + s B^T mu,  r2 = a21 M v + b21 K v + e21 N v + s B^T p
//   phase 1: r1 += a12 M l + b12 K l + e12 N^T l,  r2 += a22 M l
template <int PX, int PY, bool CV, int PH, typename R>
__device__ __forceinline__ void block_node(const cpx<R>* sx, const cpx<R>* sp, const cpx<R>* sm, int col, int la,
                                           int lb, int lane, int X0, int Y0, int n, int comp, double h,
                                           const BlockCoef& k, const R* __restrict__ ctile, cpx<R>& r1,
                                           cpx<R>& r2) {
  const int nq = 2 * n + 1;
  int lx, ly;
  node_of(PX, PY, col, la, lb, lx, ly);
  const int gx = X0 + lx, gy = Y0 + ly;
  if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) return;
  const cpx<R>* base = sx + ((ly - PY) >> 1) * kH + ((lx - PX) >> 1);
  const R* cn = CV ? ctile + ((size_t)col * kCC + coff(PX, PY)) * 64 + lane : nullptr;
  cpx<R> pm, pk, pc;
  stencil_raw<PX, PY, CV, R>(base, cn, pm, pk, pc);
  const R sM = (R)(h * h / 900.0), sK = (R)(1.0 / 90.0);
  cpx<R> Mz, Kz;
  Mz.x = sM * pm.x; Mz.y = sM * pm.y;
  Kz.x = sK * pk.x; Kz.y = sK * pk.y;
  if (PH == 0) {
    r1 = cmad<R>(r1, k.a11, Mz);
    r2 = cmad<R>(cmad<R>(r2, k.a21, Mz), k.b21, Kz);
    if (CV) r2 = cmad<R>(r2, k.e21, pc);
    // B^T p (row 2) and B^T mu (row 1) for this velocity component
    double mxx[3], gxx[3], mxy[3], gxy[3];
    mixed_cols(gx, n, h, mxx, gxx);
    mixed_cols(gy, n, h, mxy, gxy);
    const int kx0 = (gx >> 1) - 1, ky0 = (gy >> 1) - 1;
    R bpr = 0, bpi = 0, bmr = 0, bmi = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int kyy = ky0 + a;
      if (kyy < 0 || kyy > n) continue;
      const double wy = comp == 0 ? mxy[a] : gxy[a];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int kxx = kx0 + c;
        if (kxx < 0 || kxx > n) continue;
        const R wgt = (R)(wy * (comp == 0 ? gxx[c] : mxx[c]));
        const int pi = (kyy - (Y0 / 2 - 1)) * kPP + (kxx - (X0 / 2 - 1));
        const cpx<R> pv = sp[pi], mv = sm[pi];
        bpr -= wgt * pv.x; bpi -= wgt * pv.y;
        bmr -= wgt * mv.x; bmi -= wgt * mv.y;
      }
    }
    const R ks = (R)k.s;
    r1.x += ks * bmr; r1.y += ks * bmi;
    r2.x += ks * bpr; r2.y += ks * bpi;
  } else {
    r1 = cmad<R>(cmad<R>(r1, k.a12, Mz), k.b12, Kz);
    if (CV) r1 = cmad<R>(r1, k.e12, pc);
    r2 = cmad<R>(r2, k.a22, Mz);
  }
}

template <bool CV, int PH, typename R>
__device__ __forceinline__ void block_phase(const cpx<R>* sx, const cpx<R>* sp, const cpx<R>* sm, int w, int rot,
                                            int la, int lb, int lane, int X0, int Y0, int n, int comp, double h,
                                            const BlockCoef& k, const R* __restrict__ ctile, cpx<R>* r1,
                                            cpx<R>* r2) {
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    switch (class_of(w, c, rot)) {
      case 0: block_node<0, 0, CV, PH, R>(sx, sp, sm, c, la, lb, lane, X0, Y0, n, comp, h, k, ctile, r1[c], r2[c]); break;
      case 1: block_node<1, 0, CV, PH, R>(sx, sp, sm, c, la, lb, lane, X0, Y0, n, comp, h, k, ctile, r1[c], r2[c]); break;
      case 2: block_node<0, 1, CV, PH, R>(sx, sp, sm, c, la, lb, lane, X0, Y0, n, comp, h, k, ctile, r1[c], r2[c]); break;
      default: block_node<1, 1, CV, PH, R>(sx, sp, sm, c, la, lb, lane, X0, Y0, n, comp, h, k, ctile, r1[c], r2[c]); break;
    }
  }
}

// staging index (stage_idx layout) of a lane's node at colour step c
__device__ __forceinline__ int stage_at(int w, int c, int rot, int la, int lb) {
  const int cl = class_of(w, c, rot);
  int lx, ly;
  node_of(cl & 1, cl >> 1, c, la, lb, lx, ly);
  return stage_idx(lx, ly);
}

// store a staged (stage_idx layout) result tile to dst; zero on boundary nodes
template <typename R>
__device__ __forceinline__ void store_staged(cpx<R>* __restrict__ dst, const cpx<R>* st, int nq, int X0, int Y0) {
  if (threadIdx.x >= 5 * kT) return;
  const int lx = (int)threadIdx.x % kT, ly0 = (int)threadIdx.x / kT;
  const int gx = X0 + lx;
  if (gx >= nq) return;
  const bool xin = gx >= 1 && gx <= nq - 2;
  cpx<R>* d = dst + (ptrdiff_t)(Y0 + ly0) * nq + gx;
#pragma unroll
  for (int k = 0; k < kSR; ++k) {
    const int ly = ly0 + 5 * k, gy = Y0 + ly;
    if (ly >= kT || gy >= nq) break;
    const bool in = xin && gy >= 1 && gy <= nq - 2;
    d[(ptrdiff_t)5 * k * nq] = in ? st[stage_idx(lx, ly)] : cmk<cpx<R>>(0, 0);
  }
}
}  // namespace

// Velocity rows of the frequency blocks Z_j (Stokes) or G_j (Oseen): grid
// f = 2 j + comp of the batch, inputs xV [j][b][comp][(2n+1)^2] and xP
// [j][b][(n+1)^2], outputs yV (rows 1 and 2 in blocks b = 0 and 1).  tcN /
// tcNT: tile-layout tables of N and N^T (Oseen) or null.
template <typename R, bool CV>
__global__ __launch_bounds__(256, 2) void k_q2_block_vel(cpx<R>* __restrict__ yV, const cpx<R>* __restrict__ xV,
                                                      const cpx<R>* __restrict__ xP, int n,
                                                      const BlockCoef* __restrict__ bc,
                                                      const R* __restrict__ tcN, const R* __restrict__ tcNT,
                                                      int ntx, int nb, Mask mk) {
  __shared__ cpx<R> sx[4 * kSub];
  __shared__ cpx<R> sp[kPP * kPP], sm[kPP * kPP];
  int tile, f;
  if (!tile_of_block(ntx * ntx, nb, CV, tile, f)) return;
  if (mk.off(f)) return;
  const int j = f >> 1, comp = f & 1;
  const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
  const int nq = 2 * n + 1, nq2 = nq * nq, np = n + 1, np2 = np * np;
  const double h = 1.0 / n;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, rot = (int)(blockIdx.x >> 3) & 3;
  int la, lb;
  lane_ab(lane, la, lb);
  const cpx<R>* v = xV + ((size_t)(j * 2 + 0) * 2 + comp) * nq2;
  const cpx<R>* l = xV + ((size_t)(j * 2 + 1) * 2 + comp) * nq2;
  const cpx<R>* pp = xP + (size_t)(j * 2 + 0) * np2;
  const cpx<R>* pmu = xP + (size_t)(j * 2 + 1) * np2;
  // pressure patches (Q1 nodes X0/2 - 1 .. X0/2 + 24 per direction)
  for (int e = threadIdx.x; e < kPP * kPP; e += 256) {
    const int ky = Y0 / 2 - 1 + e / kPP, kx = X0 / 2 - 1 + e % kPP;
    const bool in = kx >= 0 && kx <= n && ky >= 0 && ky <= n;
    sp[e] = in ? pp[(size_t)ky * np + kx] : cmk<cpx<R>>(0, 0);
    sm[e] = in ? pmu[(size_t)ky * np + kx] : cmk<cpx<R>>(0, 0);
  }
  load_tile<R>(sx, v, nq, X0, Y0);
  const BlockCoef k = bc[j];
  const size_t toff = (size_t)tile * kTileTab;
  cpx<R> r1[9], r2[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) { r1[c] = cmk<cpx<R>>(0, 0); r2[c] = r1[c]; }
  __syncthreads();
  block_phase<CV, 0, R>(sx, sp, sm, w, rot, la, lb, lane, X0, Y0, n, comp, h, k, CV ? tcN + toff : nullptr, r1, r2);
  __syncthreads();
  load_tile<R>(sx, l, nq, X0, Y0);
  __syncthreads();
  block_phase<CV, 1, R>(sx, sp, sm, w, rot, la, lb, lane, X0, Y0, n, comp, h, k, CV ? tcNT + toff : nullptr, r1, r2);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 9; ++c) sx[stage_at(w, c, rot, la, lb)] = r1[c];
  __syncthreads();
  store_staged<R>(yV + ((size_t)(j * 2 + 0) * 2 + comp) * nq2, sx, nq, X0, Y0);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 9; ++c) sx[stage_at(w, c, rot, la, lb)] = r2[c];
  __syncthreads();
  store_staged<R>(yV + ((size_t)(j * 2 + 1) * 2 + comp) * nq2, sx, nq, X0, Y0);
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
                     const OpCoef* coef, int fpc, int nb, const R* tconv, bool forward, Mask mk) {
  const int ntx = (2 * n + 1 + kT - 1) / kT;
  const dim3 g(tile_blocks(ntx, nb)), blk(256);
  const bool cv = tconv != nullptr, pro = ec != nullptr;
#define PINTOC_SWEEP(CV, FWD, PRO)                                                                                 \
  if (cv == CV && forward == FWD && pro == PRO) {                                                                   \
    hipLaunchKernelGGL((k_q2_sweep<R, CV, FWD, PRO>), g, blk, 0, s, xo, xi, b, ec, n, h, coef, fpc, tconv, ntx, nb, \
                       mk);                                                                                         \
    return;                                                                                                         \
  }
  PINTOC_SWEEP(false, true, false)
  PINTOC_SWEEP(false, false, true)
  PINTOC_SWEEP(true, true, false)
  PINTOC_SWEEP(true, false, true)
  PINTOC_SWEEP(false, false, false)
  PINTOC_SWEEP(false, true, true)
  PINTOC_SWEEP(true, false, false)
  PINTOC_SWEEP(true, true, true)
#undef PINTOC_SWEEP
}

template <typename R>
void launch_q2_apply(hipStream_t s, cpx<R>* out, const cpx<R>* x, const cpx<R>* b, int n, double h,
                     const OpCoef* coef, int fpc, int nb, const R* tconv, Mask mk) {
  const int ntx = (2 * n + 1 + kT - 1) / kT;
  const dim3 g(tile_blocks(ntx, nb)), blk(256);
  if (tconv) hipLaunchKernelGGL((k_q2_tile_apply<R, true>), g, blk, 0, s, out, x, b, n, h, coef, fpc, tconv, ntx, nb, mk);
  else hipLaunchKernelGGL((k_q2_tile_apply<R, false>), g, blk, 0, s, out, x, b, n, h, coef, fpc, tconv, ntx, nb, mk);
}

template <typename R>
void launch_q2_residual_restrict(hipStream_t s, cpx<R>* bc, cpx<R>* side, const cpx<R>* x, const cpx<R>* b, int n,
                                 double h, const OpCoef* coef, int fpc, int nb, const R* tconv, Mask mk) {
  const int ntx = (2 * n + 1 + kT - 1) / kT;
  const dim3 g(tile_blocks(ntx, nb)), blk(256);
  if (tconv)
    hipLaunchKernelGGL((k_q2_residual_restrict<R, true>), g, blk, 0, s, bc, side, x, b, n, h, coef, fpc, tconv, ntx,
                       nb, mk);
  else
    hipLaunchKernelGGL((k_q2_residual_restrict<R, false>), g, blk, 0, s, bc, side, x, b, n, h, coef, fpc, tconv, ntx,
                       nb, mk);
  const int len = n - 1, A = len / kCT;
  if (A > 0) {
    const unsigned items = (unsigned)(2 * A * len);
    hipLaunchKernelGGL((k_q2_restrict_fix<R>), dim3((items + 255) / 256, (unsigned)nb), blk, 0, s, bc, side, n, ntx,
                       mk);
  }
}

size_t q2_restrict_side_entries(int n) { return (size_t)q2_tile_count(n) * kSide; }

template <typename R>
void launch_q2_tile_cheb(hipStream_t s, cpx<R>* xn, const cpx<R>* x, const cpx<R>* xp, const cpx<R>* b, int n,
                         double h, double g, double w, int nb, Mask mk) {
  const int ntx = (2 * n + 1 + kT - 1) / kT;
  hipLaunchKernelGGL((k_q2_tile_cheb<R>), dim3(tile_blocks(ntx, nb)), dim3(256), 0, s, xn, x, xp, b, n, h, g, w, ntx,
                     nb, mk);
}

template <typename R>
void launch_q2_block_vel(hipStream_t s, cpx<R>* yV, const cpx<R>* xV, const cpx<R>* xP, int n, int nf,
                         const BlockCoef* bc, const R* tcN, const R* tcNT, Mask mk) {
  const int ntx = (2 * n + 1 + kT - 1) / kT;
  const dim3 g(tile_blocks(ntx, 2 * nf)), blk(256);
  if (tcN) hipLaunchKernelGGL((k_q2_block_vel<R, true>), g, blk, 0, s, yV, xV, xP, n, bc, tcN, tcNT, ntx, 2 * nf, mk);
  else hipLaunchKernelGGL((k_q2_block_vel<R, false>), g, blk, 0, s, yV, xV, xP, n, bc, tcN, tcNT, ntx, 2 * nf, mk);
}

// Reorder one half (0: N, 1: N^T) of a per-node convection table (50 values
// per padded Q2 node: 25 offsets of N, then 25 of N^T) into the layout of the
// tile kernels.
void q2_tile_conv_table(int n, const double* t50, int half, double* out) {
  const int nq = 2 * n + 1, ntx = (nq + kT - 1) / kT;
  const size_t total = (size_t)ntx * ntx * kTileTab;
  for (size_t i = 0; i < total; ++i) out[i] = 0.0;
  for (int tile = 0; tile < ntx * ntx; ++tile) {
    const int X0 = (tile % ntx) * kT, Y0 = (tile / ntx) * kT;
    for (int col = 0; col < 9; ++col) {
      for (int cls = 0; cls < 4; ++cls) {
        const int PX = cls & 1, PY = cls >> 1;
        for (int lane = 0; lane < 64; ++lane) {
          int la, lb, lx, ly;
          lane_ab(lane, la, lb);
          node_of(PX, PY, col, la, lb, lx, ly);
          const int gx = X0 + lx, gy = Y0 + ly;
          if (gx < 1 || gx > nq - 2 || gy < 1 || gy > nq - 2) continue;
          int k = 0;
          for (int iy = 0; iy < wlen(PY); ++iy)
            for (int ix = 0; ix < wlen(PX); ++ix, ++k) {
              const int dx = wlo(PX) + ix, dy = wlo(PY) + iy;
              out[(((size_t)tile * 9 + col) * kCC + coff(PX, PY) + k) * 64 + lane] =
                  t50[((size_t)gy * nq + gx) * 50 + half * 25 + (dy + 2) * 5 + (dx + 2)];
            }
        }
      }
    }
  }
}

size_t q2_tile_conv_entries(int n) { return (size_t)q2_tile_count(n) * kTileTab; }

#define PINTOC_Q2T_INST(R)                                                                                       \
  template void launch_q2_sweep<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, int, double, \
                                   const OpCoef*, int, int, const R*, bool, Mask);                                  \
  template void launch_q2_apply<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, int, double, const OpCoef*,  \
                                   int, int, const R*, Mask);                                                         \
  template void launch_q2_block_vel<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, int, int,                 \
                                       const BlockCoef*, const R*, const R*, Mask);                                   \
  template void launch_q2_residual_restrict<R>(hipStream_t, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*, int,      \
                                               double, const OpCoef*, int, int, const R*, Mask);                      \
  template void launch_q2_tile_cheb<R>(hipStream_t, cpx<R>*, const cpx<R>*, const cpx<R>*, const cpx<R>*, int,        \
                                       double, double, double, int, Mask);

PINTOC_Q2T_INST(double)
PINTOC_Q2T_INST(float)

}  // namespace pintoc
