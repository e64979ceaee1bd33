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
#include "kernels.h"

namespace pintoc {

// (B^T q)_comp at Q2 node (jx, jy): -sum mix(ky,jy) gmix(kx,jx) q (comp 0) or
// -sum gmix(ky,jy) mix(kx,jx) q (comp 1).
__device__ inline double bt_node(const double* __restrict__ q, int n, double h, int jx, int jy, int comp) {
  double mxx[3], gxx[3], mxy[3], gxy[3];
  mixed_cols(jx, n, h, mxx, gxx);
  mixed_cols(jy, n, h, mxy, gxy);
  const int kx0 = (jx >> 1) - 1, ky0 = (jy >> 1) - 1, np = n + 1;
  double s = 0;
  for (int a = 0; a < 3; ++a) {
    const int ky = ky0 + a;
    if (ky < 0 || ky > n) continue;
    const double wy = comp == 0 ? mxy[a] : gxy[a];
    for (int c = 0; c < 3; ++c) {
      const int kx = kx0 + c;
      if (kx < 0 || kx > n) continue;
      const double wx = comp == 0 ? gxx[c] : mxx[c];
      s += wy * wx * q[ky * np + kx];
    }
  }
  return -s;
}

// (B v)_k at Q1 node (kx, ky), v = (vx, vy) padded Q2 grids.
__device__ inline double b_node(const double* __restrict__ vx, const double* __restrict__ vy, int n, double h,
                                int kx, int ky) {
  double mxx[5], gxx[5], mxy[5], gxy[5];
  mixed_rows(kx, n, h, mxx, gxx);
  mixed_rows(ky, n, h, mxy, gxy);
  const int nq = 2 * n + 1;
  double s = 0;
  for (int dy = 0; dy < 5; ++dy) {
    const int jy = 2 * ky + dy - 2;
    if (jy < 0 || jy >= nq) continue;
    for (int dx = 0; dx < 5; ++dx) {
      const int jx = 2 * kx + dx - 2;
      if (jx < 0 || jx >= nq) continue;
      const int j = jy * nq + jx;
      s += mxy[dy] * gxx[dx] * vx[j] + gxy[dy] * mxx[dx] * vy[j];
    }
  }
  return -s;
}

// One thread per entry g >= g0 of the canonical vector.
__global__ __launch_bounds__(256) void k_kkt_apply(const double* __restrict__ x, double* __restrict__ y, int n, int nt, double tau,
                            double beta, double nu, const double* __restrict__ conv, int g0) {
  const int nq = 2 * n + 1, nq2 = nq * nq, np = n + 1, np2 = np * np;
  const int L = 2 * nq2 + np2;
  const int g = g0 + blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y, b = blockIdx.z;
  if (g >= L) return;
  const double h = 1.0 / n;
  const double* X0 = x;                           // block 0: v, p
  const double* X1 = x + (size_t)nt * L;          // block 1: l, mu
  auto lev = [&](const double* B0, int tt) { return B0 + (size_t)tt * L; };
  double out = 0;
  if (g < 2 * nq2) {
    const int comp = g >= nq2, node = g - comp * nq2;
    const int ix = node % nq, iy = node / nq;
    if (ix > 0 && iy > 0 && ix < nq - 1 && iy < nq - 1) {
      double mx[5], kx[5], my[5], ky[5];
      q2_rows(ix, h, mx, kx);
      q2_rows(iy, h, my, ky);
      // One pass over the 25 neighbours.  Adjoint rows (b = 0):
      //   M (tau v_t + l_t - l_{t+1}) + tau nu K l_t + tau N^T l_t + tau B^T mu_t;
      // state rows (b = 1):
      //   M (v_t - v_{t-1} - tau/beta l_t) + tau nu K v_t + tau N v_t + tau B^T p_t.
      // The mass term acts on one combined field, the stiffness and convection
      // terms on the field u they differentiate (l_t, resp. v_t).
      const double* vt = lev(X0, t) + comp * nq2;
      const double* lt = lev(X1, t) + comp * nq2;
      const double* un = b == 0 ? (t + 1 < nt ? lev(X1, t + 1) + comp * nq2 : nullptr)
                                : (t > 0 ? lev(X0, t - 1) + comp * nq2 : nullptr);
      const double ca = b == 0 ? tau : 1.0, cb = b == 0 ? 1.0 : -tau / beta;   // mass field ca v_t + cb l_t - un
      const double* cn = conv ? conv + (size_t)node * 50 + (b == 0 ? 25 : 0) : nullptr;
      int cx[5];
#pragma unroll
      for (int d = 0; d < 5; ++d) cx[d] = min(max(ix + d - 2, 0), nq - 1);
      // per row: x-mass sums of the mass field (sm) and of u (su), x-stiffness
      // sums of u (sk); M = m'_y (m'_x .), K = m'_y (k'_x .) + k'_y (m'_x .)
      double mm = 0, kk = 0, cc = 0;
#pragma unroll 1
      for (int dy = 0; dy < 5; ++dy) {
        const size_t ro = (size_t)min(max(iy + dy - 2, 0), nq - 1) * nq;
        double sm = 0, sk = 0, su = 0;
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) {
          const double vv = vt[ro + cx[dx]], ll = lt[ro + cx[dx]];
          const double un_v = un ? un[ro + cx[dx]] : 0.0;
          const double u = b == 0 ? ll : vv;
          const double f = ca * vv + cb * ll - un_v;
          sm += mx[dx] * f;
          sk += kx[dx] * u;
          su += mx[dx] * u;
          if (cn) cc += cn[dy * 5 + dx] * u;
        }
        mm += my[dy] * sm;
        kk += my[dy] * sk + ky[dy] * su;
      }
      const double* pf = b == 0 ? lev(X1, t) + 2 * nq2 : lev(X0, t) + 2 * nq2;
      const double bt = bt_node(pf, n, h, ix, iy, comp);
      out = mm + tau * (nu * kk + cc) + tau * bt;
    }
  } else {
    const int k = g - 2 * nq2;
    if (k != 0) {
      const int kx = k % np, ky = k / np;
      const double* src = b == 0 ? lev(X1, t) : lev(X0, t);
      out = tau * b_node(src, src + nq2, n, h, kx, ky);
    }
  }
  y[((size_t)b * nt + t) * L + g] = out;
}

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

// Velocity rows without convection (Stokes) on LDS tiles.  A work-group owns
// 64 x 32 interior output nodes of one grid (b, t, comp) and stages the two
// fields its rows act on -- the mass field f = ca v_t + cb l_t - un and the
// differentiated field u (l_t for the adjoint rows, v_t for the state rows) --
// over the tile and a two-node halo, read once from HBM with coalesced rows.
// Thread (column, strip of 8 rows) then walks its strip keeping the x-sums
// (m' on f, k' and m' on u) of the five rows around the output row in
// registers: 10 LDS reads per output.  B^T q comes from the 3 x 3 pressure
// nodes around the output (Q1 field p_t or mu_t, read from L2).  The
// Dirichlet ring is written by k_kkt_ring.
constexpr int kVTX = 64, kVTY = 32, kVTS = 8;
constexpr int kVLX = kVTX + 4, kVLY = kVTY + 4;

__global__ __launch_bounds__(256) void k_kkt_vel_tile(const double* __restrict__ x, double* __restrict__ y, int n,
                                                      int nt, double tau, double beta, double nu, int ntx) {
  __shared__ double F[kVLY * kVLX], U[kVLY * kVLX];
  const int nq = 2 * n + 1, nq2 = nq * nq, np = n + 1, np2 = np * np;
  const int L = 2 * nq2 + np2;
  const int t = blockIdx.y, bc = blockIdx.z, b = bc >> 1, comp = bc & 1;
  const int bx = blockIdx.x % ntx, by = blockIdx.x / ntx;
  const int x0 = 1 + bx * kVTX, y0 = 1 + by * kVTY;      // first interior output node of the tile
  const double* X0 = x;
  const double* X1 = x + (size_t)nt * L;
  const double* vt = X0 + (size_t)t * L + comp * nq2;
  const double* lt = X1 + (size_t)t * L + comp * nq2;
  const double* un = b == 0 ? (t + 1 < nt ? X1 + (size_t)(t + 1) * L + comp * nq2 : nullptr)
                            : (t > 0 ? X0 + (size_t)(t - 1) * L + comp * nq2 : nullptr);
  const double ca = b == 0 ? tau : 1.0, cb2 = b == 0 ? 1.0 : -tau / beta;
  for (int e = threadIdx.x; e < kVLY * kVLX; e += blockDim.x) {
    const int ly = e / kVLX, lx = e - ly * kVLX;
    const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
    double f = 0.0, u = 0.0;
    if (gx >= 0 && gx < nq && gy >= 0 && gy < nq) {
      const size_t o = (size_t)gy * nq + gx;
      const double vv = vt[o], ll = lt[o];
      f = ca * vv + cb2 * ll - (un ? un[o] : 0.0);
      u = b == 0 ? ll : vv;
    }
    F[e] = f;
    U[e] = u;
  }
  __syncthreads();
  const int lx = threadIdx.x & (kVTX - 1), strip = threadIdx.x / kVTX;
  const int ix = x0 + lx;
  if (ix > nq - 2) return;
  const double h = 1.0 / n;
  double mx[5], kx[5], my[5], ky[5];
  q2_rows(ix, h, mx, kx);
  const double* pf = (b == 0 ? X1 : X0) + (size_t)t * L + 2 * nq2;
  const int kx0 = (ix >> 1) - 1;
  double wbx[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double m, g;
    mixed_at(kx0 + c, ix - 2 * (kx0 + c), n, h, m, g);
    wbx[c] = comp == 0 ? g : m;
  }
  double* yo = y + ((size_t)b * nt + t) * L + comp * nq2;
  const int r0 = strip * kVTS;                           // first output row of the strip (tile-local)
  double SM[5], SK[5], SU[5];
  auto sums = [&](int lr, double& sm, double& sk, double& su) {   // lr: staged row (0 = y0 - 2)
    const double* fr = F + lr * kVLX + lx;
    const double* ur = U + lr * kVLX + lx;
    sm = 0; sk = 0; su = 0;
#pragma unroll
    for (int dx = 0; dx < 5; ++dx) {
      sm += mx[dx] * fr[dx];
      sk += kx[dx] * ur[dx];
      su += mx[dx] * ur[dx];
    }
  };
#pragma unroll
  for (int d = 0; d < 4; ++d) sums(r0 + d, SM[d], SK[d], SU[d]);
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
        const int kyy = ky0 + a;
        if (kyy < 0 || kyy > n) continue;
        double m, g;
        mixed_at(kyy, iy - 2 * kyy, n, h, m, g);
        const double* row = pf + (size_t)kyy * np;
        double rs = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int kxx = kx0 + c;
          if (kxx >= 0 && kxx <= n) rs += wbx[c] * row[kxx];
        }
        bt += (comp == 0 ? m : g) * rs;
      }
      yo[(size_t)iy * nq + ix] = mm + tau * nu * kk - tau * bt;
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) { SM[d] = SM[d + 1]; SK[d] = SK[d + 1]; SU[d] = SU[d + 1]; }
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

void launch_kkt_apply(hipStream_t s, const double* x, double* y, int n, int nt, double tau, double beta, double nu,
                      const double* conv) {
  const int nq = 2 * n + 1, L = 2 * nq * nq + (n + 1) * (n + 1);
  if (conv) {                               // Oseen: every entry per thread
    hipLaunchKernelGGL(k_kkt_apply, dim3((L + 255) / 256, nt, 2), dim3(256), 0, s, x, y, n, nt, tau, beta, nu, conv,
                       0);
    return;
  }
  // Stokes: velocity rows on LDS tiles (and the Dirichlet ring), pressure rows per entry
  const int ntx = (nq - 2 + kVTX - 1) / kVTX, nty = (nq - 2 + kVTY - 1) / kVTY;
  hipLaunchKernelGGL(k_kkt_vel_tile, dim3(ntx * nty, nt, 4), dim3(256), 0, s, x, y, n, nt, tau, beta, nu, ntx);
  hipLaunchKernelGGL(k_kkt_ring, dim3((4 * (nq - 1) + 255) / 256, nt, 4), dim3(256), 0, s, y, n, nt);
  const int g0 = 2 * nq * nq, np2 = (n + 1) * (n + 1);
  hipLaunchKernelGGL(k_kkt_apply, dim3((np2 + 255) / 256, nt, 2), dim3(256), 0, s, x, y, n, nt, tau, beta, nu, conv,
                     g0);
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
