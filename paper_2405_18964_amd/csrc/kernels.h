// Launchers of the pintoc device kernels (internal to the library).
// Every batched per-frequency launcher takes a Mask: grids of frequencies
// whose mask entry is 0 are skipped (kAll: every grid active).
#pragma once
#include <vector>

#include "common.h"

namespace pintoc {

constexpr Mask kAll{nullptr, 1};

// time FFT (fft_kernels.hip)
template <typename R>
void launch_time_fft_fwd(hipStream_t s, const double* r, cpx<R>* V, cpx<R>* P, int nt, int L, int nq2, int np2,
                         const double2* tw, const double2* tj, double tau, int mode);
template <typename R>
void launch_time_fft_inv(hipStream_t s, const cpx<R>* V, const cpx<R>* P, double* z, int nt, int L, int nq2,
                         int np2, const double2* tw, const double2* tj, double tau, int mode);

// per-frequency operators and multigrid pieces (mg_kernels.hip).  For Q2
// grids ``conv`` is a convection table in the tile layout of
// q2_tile_conv_table (one operator half, scaled by coef.eta) stored in the
// grids' precision R; for Q1 grids it is the per-node FP64 table of 9 + 9
// values (coef.eta, coef.etat).
template <typename R>
void launch_tile_sweep(hipStream_t s, bool q2, cpx<R>* xo, const cpx<R>* xi, const cpx<R>* b, const cpx<R>* ec,
                       int n, double h, const OpCoef* coef, int fpc, int nb, const void* conv, bool forward,
                       Mask mk);
// Multicolour Gauss-Seidel over whole grids (one launch per colour, in place;
// forward: colours 0..C-1, backward C-1..0).  conv: Q2 per-node table of the
// level (50 values per node: N then N^T, scaled by coef.eta / coef.etat) or null.
template <typename R>
void launch_colour_sweep(hipStream_t s, bool q2, cpx<R>* x, const cpx<R>* b, int n, double h, const OpCoef* coef,
                         int fpc, int nb, const double* conv, bool forward, Mask mk);
// x = t + P ec (prolongation from the level with n / 2 elements per side)
template <typename R>
void launch_prolong_add(hipStream_t s, bool q2, cpx<R>* x, const cpx<R>* t, const cpx<R>* ec, int n, int nb,
                        Mask mk);
template <typename R>
void launch_q1_residual(hipStream_t s, cpx<R>* r, const cpx<R>* x, const cpx<R>* b, int n, double h,
                        const OpCoef* coef, int fpc, int nb, const double* conv, Mask mk);
template <typename R>
void launch_apply(hipStream_t s, bool q2, cpx<R>* y, const cpx<R>* x, int n, double h, const OpCoef* coef, int fpc,
                  int nb, const void* conv, Mask mk);
template <typename R>
void launch_q1_restrict(hipStream_t s, cpx<R>* bc, const cpx<R>* rf, int nc, int nb, Mask mk);
template <typename R>
void launch_coarse(hipStream_t s, bool q2, cpx<R>* x, const cpx<R>* b, const double2* inv, int fpc, int nb, Mask mk);
// the rest of a Q2 V-cycle from level n0 <= kQ2SmallN down to N = 2 in one
// launch, one work-group per grid; x0: initial iterate or null (zero); tconv:
// the convection table of q2_small_conv_table (scaled by coef.eta) in the
// grids' precision, or null; coef[l cstride + set]: coefficients of the l-th
// level below n0 (l = 0: n0)
constexpr int kQ2SmallN = 16;
template <typename R>
void launch_q2_small_vcycle(hipStream_t s, cpx<R>* x, const cpx<R>* x0, const cpx<R>* b, int n0, const OpCoef* coef,
                            int cstride, int fpc, const double2* inv, const R* tconv, int nb, Mask mk);
size_t q2_small_conv_entries(int n0);
void q2_small_conv_table(int n0, const std::vector<const double*>& tabs, int half, double* out);
// the same for the unconstrained Q1 hierarchies (n0 <= kQ1SmallN), whose
// operator is the same on every level (coef: the sets of level n0)
constexpr int kQ1SmallN = 16;
template <typename R>
void launch_q1_small_vcycle(hipStream_t s, cpx<R>* x, const cpx<R>* x0, const cpx<R>* b, int n0, const OpCoef* coef,
                            int fpc, const double2* inv, int nb, Mask mk);
template <typename R>
void launch_cheb(hipStream_t s, bool q2, cpx<R>* xn, const cpx<R>* x, const cpx<R>* xp, const cpx<R>* b, int n,
                 double h, double g, double w, int first, int nb, Mask mk);
template <typename R>
void launch_schur_combine_pin(hipStream_t s, cpx<R>* out, const cpx<R>* yK, const cpx<R>* yM, const double2* ab,
                              int fpc, int nn, int nb, Mask mk);

// Q2 tile kernels (q2_tiles.hip)
template <typename R>
void launch_q2_sweep(hipStream_t s, cpx<R>* xo, const cpx<R>* xi, const cpx<R>* b, const cpx<R>* ec, int n, double h,
                     const OpCoef* coef, int fpc, int nb, const R* tconv, bool forward, Mask mk);
template <typename R>
void launch_q2_apply(hipStream_t s, cpx<R>* out, const cpx<R>* x, const cpx<R>* b, int n, double h,
                     const OpCoef* coef, int fpc, int nb, const R* tconv, Mask mk);
template <typename R>
void launch_q2_block_vel(hipStream_t s, cpx<R>* yV, const cpx<R>* xV, const cpx<R>* xP, int n, int nf,
                         const BlockCoef* bc, const R* tcN, const R* tcNT, Mask mk);
// bc = P^T (b - A x) on the coarse grid of side n + 1 without storing the fine
// residual; side: q2_restrict_side_entries(n) * nb complex entries of scratch
template <typename R>
void launch_q2_residual_restrict(hipStream_t s, cpx<R>* bc, cpx<R>* side, const cpx<R>* x, const cpx<R>* b, int n,
                                 double h, const OpCoef* coef, int fpc, int nb, const R* tconv, Mask mk);
size_t q2_restrict_side_entries(int n);
// Chebyshev step (not the first) for the Q2 mass matrix on LDS tiles
template <typename R>
void launch_q2_tile_cheb(hipStream_t s, cpx<R>* xn, const cpx<R>* x, const cpx<R>* xp, const cpx<R>* b, int n,
                         double h, double g, double w, int nb, Mask mk);
size_t q2_tile_conv_entries(int n);
void q2_tile_conv_table(int n, const double* t50, int half, double* out);

// all-at-once matrix, rhs, FP64 vector kernels (kkt_kernels.hip)
// convT: Oseen convection entries of the finest grid, entry-major ([50][nq^2]:
// N at entries 0..24, N^T at 25..49); nullptr for Stokes
void launch_kkt_apply(hipStream_t s, const double* x, double* y, int n, int nt, double tau, double beta, double nu,
                      const double* convT);
void launch_assemble_rhs(hipStream_t s, const double* vd, double* b, int n, int nt, double tau);
void launch_rhs_data(hipStream_t s, const double* vd, const double* f, const double* hb, const double* v0, double* b,
                     int n, int nt, double tau, double nu, const double* conv);
void launch_scale_canon(hipStream_t s, double* y, const double* x, int n, int nt, double sv, double sp);
void launch_mdot(hipStream_t s, const double* V, size_t ld, int k, const double* w, size_t n, double* part,
                 double* out);
void launch_mgs_update(hipStream_t s, double* w, const double* V, size_t ld, int k, const double* c, size_t n);
void launch_axpby(hipStream_t s, double* y, const double* x, double a, double b, size_t n);
void launch_axpbypcz(hipStream_t s, double* y, const double* x, const double* z, double a, double b, double c,
                     size_t n);
void launch_lincomb_add(hipStream_t s, double* y, const double* Z, size_t ld, int k, const double* c, size_t n);
void launch_to_f32(hipStream_t s, float* y, const double* x, size_t n);
void launch_lincomb_add_f32(hipStream_t s, double* y, const float* Z, size_t ld, int k, const double* c, size_t n);
void launch_fill_zero(hipStream_t s, void* p, size_t bytes);

// outer Krylov method in the frequency domain (freq_kernels.hip)
void launch_freq_scale(hipStream_t s, double2* y, const double2* x, const double* f, int nf, int segV, int segP);
template <typename R>
void launch_freq_convert(hipStream_t s, const double2* xo, cpx<R>* V, cpx<R>* P, double2* yo, int nf, int nq2,
                         int np2, const double2* tj, double tau, int mode, int dir);
// y += the corner term of A^ applied to x (tmp: 8 (2N+1)^2 doubles)
void launch_freq_corner(hipStream_t s, double2* yV, const double2* xV, double* tmp, const double* sj, int n, int nf,
                        int nt);

// per-frequency GMRES vector operations (inner_kernels.hip)
template <typename R>
void launch_fdot(hipStream_t s, const cpx<R>* bV, const cpx<R>* bP, size_t ldV, size_t ldP, int k, const cpx<R>* wV,
                 const cpx<R>* wP, int segV, int segP, int nf, double2* part, double2* out, Mask mk);
size_t fdot_part_entries(int segV, int segP, int nf);
template <typename R>
void launch_fupdate(hipStream_t s, cpx<R>* wV, cpx<R>* wP, const cpx<R>* bV, const cpx<R>* bP, size_t ldV,
                    size_t ldP, int k, const double2* c, int segV, int segP, int nf, double sign, Mask mk);
template <typename R>
void launch_fdot_lag(hipStream_t s, const cpx<R>* bV, const cpx<R>* bP, size_t ldV, size_t ldP, int k,
                     const cpx<R>* uV, const cpx<R>* uP, const cpx<R>* wV, const cpx<R>* wP, int segV, int segP,
                     int nf, double2* part, double2* out, Mask mk);
template <typename R>
void launch_fupdate_lag(hipStream_t s, cpx<R>* bV, cpx<R>* bP, size_t ldV, size_t ldP, int k, const double2* cs,
                        const double2* cc, const double2* ag, int segV, int segP, int nf, double2* part,
                        double2* out, Mask mk);
size_t lag_part_entries(int segV, int segP, int nf, int m);
template <typename R>
void launch_fscale(hipStream_t s, cpx<R>* yV, cpx<R>* yP, const cpx<R>* xV, const cpx<R>* xP, const double2* a,
                   int segV, int segP, int nf, Mask mk);
template <typename R>
void launch_unpin_copy(hipStream_t s, cpx<R>* dst, const cpx<R>* src, int nn, int nb, Mask mk);
// y = a_j y + b_j x1 + c_j x2 per frequency (coef: a[nf], b[nf], c[nf]; x2 may be null)
template <typename R>
void launch_fcomb3(hipStream_t s, cpx<R>* yV, cpx<R>* yP, const cpx<R>* x1V, const cpx<R>* x1P, const cpx<R>* x2V,
                   const cpx<R>* x2P, const double* coef, int segV, int segP, int nf, Mask mk);
template <typename Rd, typename Rs>
void launch_convert(hipStream_t s, cpx<Rd>* d, const cpx<Rs>* src, size_t n);

// frequency blocks and the Oseen preconditioner pieces (oseen_kernels.hip)
template <typename R>
void launch_block_mat(hipStream_t s, cpx<R>* yV, cpx<R>* yP, const cpx<R>* xV, const cpx<R>* xP, int n, int nf,
                      const BlockCoef* bc, const R* tcN, const R* tcNT, Mask mk);
// per-frequency parameters ftau, fbeta, fnu: one entry per kept frequency
template <typename R>
void launch_schur_rhs(hipStream_t s, cpx<R>* out, const cpx<R>* in, const cpx<R>* y1, const cpx<R>* y2, int n,
                      int nf, const double* ftau, Mask mk);
template <typename R>
void launch_oseen_hp(hipStream_t s, cpx<R>* U, const cpx<R>* zz, int n, int nf, const double2* dj, const double* ftau,
                     const double* fbeta, const double* fnu, const double* conv, Mask mk);
template <typename R>
void launch_block_copy(hipStream_t s, cpx<R>* V, cpx<R>* X, int n, int nf, int b, int dir, Mask mk);
template <typename R>
void launch_combine3(hipStream_t s, cpx<R>* out, const cpx<R>* A, const cpx<R>* B, const cpx<R>* C, double c0,
                     double c1, double c2, const double* c1f, size_t n, int seg, Mask mk);

}  // namespace pintoc
