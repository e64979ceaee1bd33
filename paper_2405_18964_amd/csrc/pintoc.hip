// Host side of the pintoc library: problem set-up, workspace plan, the
// block-circulant preconditioner (sections 3-4) and the outer flexible GMRES
// (section 3.4).  Every arithmetic step on vectors runs in the kernels of
// fft_kernels.hip, mg_kernels.hip and kkt_kernels.hip; the host only holds
// scalars (per-frequency constants, Hessenberg matrices, coarsest-grid
// inverses computed once at set-up).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pintoc.h"
#include "kernels.h"

using namespace pintoc;
using cd = std::complex<double>;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;
static int fail(int code, const std::string& msg) { g_err = msg; return code; }
#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(PINTOC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------ timing probe
// Ring of HIP event pairs around launches of the dominant kernel.
// Algorithmic bytes of each timed launch are kept beside its events.
struct Probe {
  static constexpr int kCap = 4096;
  std::vector<hipEvent_t> e0, e1;
  std::vector<double> bytes;
  long count = 0;
  bool on = false;
  int create() {
    if (!e0.empty()) return PINTOC_OK;
    e0.resize(kCap); e1.resize(kCap); bytes.assign(kCap, 0.0);
    for (int i = 0; i < kCap; ++i) {
      if (hipEventCreate(&e0[i]) != hipSuccess || hipEventCreate(&e1[i]) != hipSuccess) return PINTOC_EHIP;
    }
    return PINTOC_OK;
  }
  ~Probe() {
    for (auto e : e0) (void)hipEventDestroy(e);
    for (auto e : e1) (void)hipEventDestroy(e);
  }
};

// ------------------------------------------------------------ multigrid plan
struct MGPlan {
  bool q2 = true;
  int nlev = 0;
  int N = 0;            // finest n
  int nb = 0;           // grids in the batch
  int fpc = 1;          // grids per coefficient set
  int ncoef = 0;
  std::vector<OpCoef> coef_h;          // finest level; eta scales N, etat scales N^T
  std::vector<double> visc;            // [level][set]: real diffusion coefficient replacing gamma (empty: gamma;
                                       // Q1 plans keep one operator on every level)
  std::vector<OpCoef> coef_dev_h;      // as uploaded, [level][set]: Q2 tile kernels apply eta to the plan's one table
  std::vector<double2> inv_h;          // coarsest inverses, per coefficient set
  OpCoef* coef = nullptr;              // device, [level][set]
  double2* inv = nullptr;              // device
  std::vector<const void*> conv;       // per level (device; Q2: tile layout in the grids' precision) or null
  const void* sconv = nullptr;         // Q2 small levels n <= sconv_n: per-node table (grids' precision) or null
  int sconv_n = 0;
  // per-level device buffers (complex, precision-typed): b, x (level >= 1),
  // t (second iterate buffer of the out-of-place smoother), r (residual)
  std::vector<void*> b, x, r, t;
  // global multicolour smoother (PINTOC_SMOOTHER_GLOBAL): coefficient sets
  // as defined ([level][set], eta on N and etat on N^T) and per-level 50-entry
  // Q2 convection tables (null without convection)
  bool global = false;
  std::vector<OpCoef> coefg_h;
  OpCoef* coefg = nullptr;
  std::vector<const double*> conv50;
  const OpCoef* coefgl(int l) const { return coefg + (size_t)l * ncoef; }
  Probe* probe = nullptr;              // times the finest-level pre-smoothing sweeps when on
  Probe* probe_post = nullptr;         // times the finest-level post-smoothing sweeps when on
  int fpj = 1;                         // grids per frequency in the batch
  const int* mask = nullptr;           // per-frequency activity (inner GMRES), or null
  int active = 0;                      // grids of the batch that the mask leaves active
  Mask mk() const { return Mask{mask, fpj}; }
  const OpCoef* coefl(int l) const { return coef + (size_t)l * ncoef; }
  // coefficient set c on level l (host)
  OpCoef level_coef(int set, int l) const {
    OpCoef r = coef_h[set];
    if (!visc.empty()) r.gamma = make_double2(visc[(size_t)l * ncoef + set], 0.0);
    return r;
  }
  int n(int l) const { return N >> l; }
  size_t nodes(int l) const {
    const size_t m = q2 ? (size_t)(2 * n(l) + 1) : (size_t)(n(l) + 1);
    return m * m;
  }
};

// Captured block-preconditioner applications (options.graphs), keyed by the
// buffers and the mask they were captured with.
struct GraphKey {
  const void *inV, *inP, *outV, *outP;
  const int* mask;
  int rsize;
  bool operator==(const GraphKey& o) const {
    return inV == o.inV && inP == o.inP && outV == o.outV && outP == o.outP && mask == o.mask && rsize == o.rsize;
  }
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
};

// One problem of a group (a lone problem is a group of one).  Its kept
// frequencies are f0 .. f0 + nf - 1 of the group's batch, its twiddles start
// at tw0; nu is the viscosity of the unit-square equivalent.  The outer Krylov
// vectors are the member's own.
struct Member {
  int nt = 0, nf = 0, f0 = 0, tw0 = 0;
  double T = 0, tau = 0, nu = 0, beta = 0;
  int64_t n_all = 0;
  double *Vk = nullptr, *Zk = nullptr, *rvec = nullptr, *xtmp = nullptr;
  float* Zk32 = nullptr;                // FP32 basis (options.z_fp32; then Zk is null and xtmp holds z)
};

struct pintoc_problem {
  pintoc_problem_desc d{};
  std::vector<Member> mem;              // one entry for a lone problem
  bool group = false;                   // created by pintoc_group_create
  std::vector<int> mem_on, freq_on;     // members (and their frequencies) taking part in the current application
  pintoc_options o{};
  std::vector<double> wind;
  double tau = 0;
  int nf = 0, L = 0, nq2 = 0, np2 = 0;
  int64_t n_all = 0;
  size_t csize = 16;                    // bytes per complex entry of the inner solves
  // host tables
  std::vector<double2> tw_h, tj_h, ab_h;
  // device tables / buffers (carved from the workspace)
  void* ws = nullptr;
  size_t ws_bytes = 0, need = 0;
  double2 *tw = nullptr, *tj = nullptr, *ab = nullptr;
  // frequency vectors (precision of the inner solves): S = transformed residual,
  // X = block solution, Zt/U = GMRES temporaries, B = inner Krylov basis
  void *Vb = nullptr, *Vx = nullptr, *Pb = nullptr, *Px = nullptr;
  void *ZtV = nullptr, *ZtP = nullptr, *UV = nullptr, *UP = nullptr, *BV = nullptr, *BP = nullptr;
  void *Ptmp = nullptr, *PxK = nullptr, *PxM = nullptr, *PxM2 = nullptr;
  double2 *cj = nullptr, *hdev = nullptr, *h2dev = nullptr, *ydev = nullptr, *fpart = nullptr;
  // lagged Gram-Schmidt: dot sweep results, update coefficients (s_i, c_i per
  // frequency; alpha and gamma), norms of the once-projected vectors
  double2 *lagOut = nullptr, *lagCS = nullptr, *lagCC = nullptr, *lagAG = nullptr, *lagRho = nullptr;
  std::vector<double2> cj_h;
  int segV = 0, segP = 0;
  MGPlan mgW, mgK;
  // block coefficients of Z_j (Stokes) or G_j (Oseen), per kept frequency
  std::vector<BlockCoef> bc_h;
  BlockCoef* bc = nullptr;
  // Oseen: convection tables (host copies and device), Q_j / Q_j^H multigrid,
  // operator tables of the Uzawa steps and the Schur step
  std::vector<std::vector<double>> conv2_h;   // per level, 50 per Q2 node
  std::vector<double> conv1_h;                // finest Q1 grid, 18 per node
  std::vector<std::vector<double>> tconv_h[2];  // per level below the coarsest: N, N^T in tile layout
  std::vector<void*> tconv[2];                 // device, in the inner precision (double or float entries)
  std::vector<double> sconv_h[2];              // levels n <= kQ2SmallN (above the coarsest): per-node layout
  void* sconv[2] = {nullptr, nullptr};         // device, in the inner precision
  int sconv_n = 0;                             // finest level of the small tables
  double* conv50 = nullptr;                   // finest level, 50 per node (block matrices)
  std::vector<double> conv50t_h;              // finest level entry-major: entry e of node g at e nq^2 + g
  double* conv50t = nullptr;                  // device copy (all-at-once matrix)
  std::vector<double*> conv50l;               // every level, 50 per node (global smoother only; [0] = conv50)
  double* conv1 = nullptr;
  MGPlan mgQ, mgQH;
  int* maskd = nullptr;                 // device mask of the batched inner GMRES
  std::vector<int> mask_h;
  const int* cur_mask = nullptr;       // mask in force for the current block operations
  Mask mk(int fpj) const { return Mask{cur_mask, fpj}; }
  std::vector<OpCoef> cpsi_h, cpsih_h;
  OpCoef *cpsi = nullptr, *cpsih = nullptr, *cscal = nullptr;   // cscal: [tau M, tau/beta M, M][j]
  std::vector<double2> dj_h;
  double2 *dj = nullptr, *abO = nullptr;                          // abO[j] = -1/tau^2
  std::vector<OpCoef> cscal_h[3];
  std::vector<double2> abO_h;
  // per kept frequency: its member's tau, 1/tau, beta, nu
  std::vector<double> ftau_h, finvtau_h, fbeta_h, fnu_h;
  double *ftau = nullptr, *finvtau = nullptr, *fbeta = nullptr, *fnu = nullptr;
  void *B1 = nullptr, *B2 = nullptr, *X1 = nullptr, *X2 = nullptr, *T1 = nullptr, *T2 = nullptr, *Rb = nullptr;
  void *C1 = nullptr, *C2 = nullptr, *Pt = nullptr, *Ub = nullptr;
  Probe probe, probe_post;
  // device time per phase of a solve: pairs of HIP events on the solve's
  // stream, summed when the solve ends
  struct PhaseTimer {
    std::vector<hipEvent_t> e0, e1;
    std::vector<int> phase;
    size_t used = 0;
    bool on = false;
    ~PhaseTimer() {
      for (auto e : e0) (void)hipEventDestroy(e);
      for (auto e : e1) (void)hipEventDestroy(e);
    }
  } pt;
  // modelled bytes: the whole solve so far, and the parts of one application
  double bytes_acc = 0.0;
  double model_fft = 0.0, model_block = 0.0, model_bmat = 0.0, model_fvec = 0.0, model_canon = 0.0;
  std::vector<long> its_acc;           // inner GMRES iterations per frequency, summed over a solve
  // inner statistics
  long inner_its_sum = 0, inner_blocks = 0;
  int inner_its_max = 0;
  std::vector<int> last_its;
  // outer FGMRES
  double *Vk = nullptr, *Zk = nullptr, *rvec = nullptr, *xtmp = nullptr;
  double *dd = nullptr, *dd2 = nullptr, *part = nullptr;
  bool bound = false;
  double side = 1.0;                    // side of the square domain (section 5: [-1, 1]^2 has 2)
  // frequency-domain FGMRES: outer vector length (reals), b~, scalings s_j and
  // 1/s_j, scratch of the corner term, the G_j coefficients (Stokes)
  int64_t nF = 0;
  double *fb = nullptr, *fsc = nullptr, *fisc = nullptr, *ftmp = nullptr;
  std::vector<double> fsc_h, fisc_h;
  std::vector<BlockCoef> gc_h;
  BlockCoef* gcoef = nullptr;
  double* dscale = nullptr;             // one canonical vector for the domain scaling (side != 1 only)
  int scratch_dev = -1;                 // device whose static scratch is bound (pintoc_bind_scratch), or -1
  // side stream of the Stokes preconditioner (pressure part beside the
  // velocity multigrid) and its fork/join events; default priority
  hipStream_t pstream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<GraphEntry> graphs;       // captured block-preconditioner applications (options.graphs)
  // statistics
  int precond_apps = 0;
  // a solve paused at a restart boundary (pintoc_solve_stats.cycle_budget):
  // its vectors stay in device memory (x and b are the caller's, the rest is
  // rebuilt from them), the scalars that carry over are kept here
  struct Paused {
    bool on = false;
    const double* b = nullptr;
    double* x = nullptr;
    int its = 0;
    double bnorm = 0, res0 = 0;
    std::vector<double> hist;
    std::chrono::steady_clock::duration elapsed{};
    double phase[PINTOC_NPHASES] = {};
  } paused;
};

// -------------------------------------------------------- small host helpers
static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Dense complex inverse by Gauss-Jordan elimination with partial pivoting.
static bool invert(std::vector<cd>& A, int n) {
  std::vector<cd> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(A[r * n + c]) > std::abs(A[p * n + c])) p = r;
    if (std::abs(A[p * n + c]) == 0.0) return false;
    if (p != c)
      for (int k = 0; k < n; ++k) { std::swap(A[p * n + k], A[c * n + k]); std::swap(I[p * n + k], I[c * n + k]); }
    const cd piv = A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] /= piv; I[c * n + k] /= piv; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const cd f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; I[r * n + k] -= f * I[c * n + k]; }
    }
  }
  A.swap(I);
  return true;
}

static cd toc(double2 v) { return cd(v.x, v.y); }

// Coarsest (n = 2) operator alpha M + gamma K (+ eta N + etat N^T) as a dense
// matrix and its inverse.  Q2: the 9 interior nodes of the padded 5x5 grid.
// Q1: the 9 nodes of the 3x3 grid with node 0 removed (8x8).
static bool coarse_inverse(bool q2, const OpCoef& c, const std::vector<double>* conv, std::vector<double2>& out) {
  const int n = 2;
  const double h = 1.0 / n;
  if (q2) {
    std::vector<cd> A(81, 0.0);
    for (int r = 0; r < 9; ++r) {
      const int ix = 1 + r % 3, iy = 1 + r / 3;
      double mx[5], kx[5], my[5], ky[5];
      q2_rows(ix, h, mx, kx);
      q2_rows(iy, h, my, ky);
      for (int q = 0; q < 9; ++q) {
        const int jx = 1 + q % 3, jy = 1 + q / 3, dx = jx - ix + 2, dy = jy - iy + 2;
        if (dx < 0 || dx > 4 || dy < 0 || dy > 4) continue;
        cd v = toc(c.alpha) * (mx[dx] * my[dy]) + toc(c.gamma) * (kx[dx] * my[dy] + mx[dx] * ky[dy]);
        if (conv) {
          const double* cn = conv->data() + (size_t)(iy * 5 + ix) * 50;
          v += toc(c.eta) * cn[dy * 5 + dx] + toc(c.etat) * cn[25 + dy * 5 + dx];
        }
        A[r * 9 + q] = v;
      }
    }
    if (!invert(A, 9)) return false;
    for (auto& v : A) out.push_back(make_double2(v.real(), v.imag()));
  } else {
    std::vector<cd> A(64, 0.0);
    for (int r = 1; r < 9; ++r) {
      const int ix = r % 3, iy = r / 3;
      double mx[3], kx[3], my[3], ky[3];
      q1_rows(ix, n, h, mx, kx);
      q1_rows(iy, n, h, my, ky);
      for (int q = 1; q < 9; ++q) {
        const int jx = q % 3, jy = q / 3, dx = jx - ix + 1, dy = jy - iy + 1;
        if (dx < 0 || dx > 2 || dy < 0 || dy > 2) continue;
        cd v = toc(c.alpha) * (mx[dx] * my[dy]) + toc(c.gamma) * (kx[dx] * my[dy] + mx[dx] * ky[dy]);
        if (conv) {
          const double* cn = conv->data() + (size_t)(iy * 3 + ix) * 18;
          v += toc(c.eta) * cn[dy * 3 + dx] + toc(c.etat) * cn[9 + dy * 3 + dx];
        }
        A[(r - 1) * 8 + (q - 1)] = v;
      }
    }
    if (!invert(A, 8)) return false;
    for (auto& v : A) out.push_back(make_double2(v.real(), v.imag()));
  }
  return true;
}

static OpCoef mkcoef(cd a, cd g, cd e = 0.0, cd et = 0.0) {
  OpCoef c;
  c.alpha = make_double2(a.real(), a.imag());
  c.gamma = make_double2(g.real(), g.imag());
  c.eta = make_double2(e.real(), e.imag());
  c.etat = make_double2(et.real(), et.imag());
  return c;
}

// ------------------------------------------------------------ workspace plan
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T> T* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  }
};

static void plan_mg_buffers(MGPlan& m, Carver& cv, size_t csize) {
  m.b.assign(m.nlev, nullptr);
  m.x.assign(m.nlev, nullptr);
  m.r.assign(m.nlev, nullptr);
  m.t.assign(m.nlev, nullptr);
  for (int l = 0; l < m.nlev; ++l) {
    const size_t bytes = m.nodes(l) * m.nb * csize;
    if (l > 0) {
      m.b[l] = cv.take<char>(bytes);
      m.x[l] = cv.take<char>(bytes);
    }
    if (l + 1 < m.nlev) {
      // Q2 levels restrict without storing the residual: r holds the shared partial sums only
      m.r[l] = cv.take<char>(m.q2 ? q2_restrict_side_entries(m.n(l)) * m.nb * csize : bytes);
      m.t[l] = cv.take<char>(bytes);
    }
  }
  m.coef = cv.take<OpCoef>(sizeof(OpCoef) * m.ncoef * m.nlev);
  m.inv = cv.take<double2>(sizeof(double2) * m.inv_h.size());
  m.coefg = m.global ? cv.take<OpCoef>(sizeof(OpCoef) * m.coefg_h.size()) : nullptr;
}

static void carve(pintoc_problem* p, char* base) {
  Carver cv{base};
  const int nf = p->nf;
  p->tw = cv.take<double2>(sizeof(double2) * p->tw_h.size());
  p->ftau = cv.take<double>(sizeof(double) * nf);
  p->finvtau = cv.take<double>(sizeof(double) * nf);
  p->fbeta = cv.take<double>(sizeof(double) * nf);
  p->fnu = cv.take<double>(sizeof(double) * nf);
  p->tj = cv.take<double2>(sizeof(double2) * nf);
  p->ab = cv.take<double2>(sizeof(double2) * nf);
  const size_t vbytes = (size_t)4 * nf * p->nq2 * p->csize;
  const size_t pbytes = (size_t)2 * nf * p->np2 * p->csize;
  p->cj = cv.take<double2>(sizeof(double2) * nf);
  p->Vb = cv.take<char>(vbytes);
  p->Vx = cv.take<char>(vbytes);
  p->Pb = cv.take<char>(pbytes);
  p->Px = cv.take<char>(pbytes);
  p->Ptmp = cv.take<char>(pbytes);
  p->PxK = cv.take<char>(pbytes);
  p->PxM = cv.take<char>(pbytes);
  p->PxM2 = cv.take<char>(pbytes);
  if (p->o.inner != PINTOC_INNER_LINEAR) {
    // inner GMRES: the Arnoldi basis; inner MINRES: its seven block vectors
    const int mi = p->o.inner == PINTOC_INNER_MINRES ? 6 : p->o.inner_restart;
    p->ZtV = cv.take<char>(vbytes);
    p->ZtP = cv.take<char>(pbytes);
    p->UV = cv.take<char>(vbytes);
    p->UP = cv.take<char>(pbytes);
    p->BV = cv.take<char>(vbytes * (mi + 1));
    p->BP = cv.take<char>(pbytes * (mi + 1));
    p->hdev = cv.take<double2>(sizeof(double2) * (mi + 1) * nf);
    p->h2dev = cv.take<double2>(sizeof(double2) * (mi + 1) * nf);
    p->ydev = cv.take<double2>(sizeof(double2) * (mi + 1) * nf);
    p->fpart = cv.take<double2>(sizeof(double2) * std::max(fdot_part_entries(p->segV, p->segP, nf),
                                                           lag_part_entries(p->segV, p->segP, nf, mi)));
    p->lagOut = cv.take<double2>(sizeof(double2) * (2 * mi + 2) * nf);
    p->lagCS = cv.take<double2>(sizeof(double2) * mi * nf);
    p->lagCC = cv.take<double2>(sizeof(double2) * mi * nf);
    p->lagAG = cv.take<double2>(sizeof(double2) * 2 * nf);
    p->lagRho = cv.take<double2>(sizeof(double2) * nf);
  }
  p->bc = cv.take<BlockCoef>(sizeof(BlockCoef) * nf);
  p->maskd = cv.take<int>(sizeof(int) * nf);
  if (p->d.flow == PINTOC_OSEEN) {
    p->conv50 = cv.take<double>(sizeof(double) * p->conv2_h[0].size());
    p->conv50t = cv.take<double>(sizeof(double) * p->conv50t_h.size());
    for (int hf = 0; hf < 2; ++hf) {
      p->tconv[hf].assign(p->tconv_h[hf].size(), nullptr);
      for (size_t l = 0; l < p->tconv_h[hf].size(); ++l)
        p->tconv[hf][l] = cv.take<char>(p->csize / 2 * p->tconv_h[hf][l].size());
      p->sconv[hf] = p->sconv_h[hf].empty() ? nullptr : cv.take<char>(p->csize / 2 * p->sconv_h[hf].size());
    }
    p->conv1 = cv.take<double>(sizeof(double) * p->conv1_h.size());
    p->cpsi = cv.take<OpCoef>(sizeof(OpCoef) * nf);
    p->cpsih = cv.take<OpCoef>(sizeof(OpCoef) * nf);
    p->cscal = cv.take<OpCoef>(sizeof(OpCoef) * 3 * nf);
    p->dj = cv.take<double2>(sizeof(double2) * nf);
    p->abO = cv.take<double2>(sizeof(double2) * nf);
    const size_t hb = (size_t)2 * nf * p->nq2 * p->csize;    // one velocity block: [j][comp]
    for (void** q : {&p->B1, &p->B2, &p->X1, &p->X2, &p->T1, &p->T2, &p->Rb, &p->C1, &p->C2}) *q = cv.take<char>(hb);
    p->Pt = cv.take<char>(pbytes);
    p->Ub = cv.take<char>(pbytes);
    for (size_t l = 0; l < p->tconv[0].size(); ++l) { p->mgQ.conv[l] = p->tconv[0][l]; p->mgQH.conv[l] = p->tconv[1][l]; }
    if (p->o.smoother == PINTOC_SMOOTHER_GLOBAL) {
      // per-node tables of every level the global sweep visits (the finest is conv50)
      p->conv50l.assign(p->conv2_h.size(), nullptr);
      p->conv50l[0] = p->conv50;
      for (size_t l = 1; l < p->conv2_h.size(); ++l) p->conv50l[l] = cv.take<double>(sizeof(double) * p->conv2_h[l].size());
      p->mgQ.conv50.assign(p->conv50l.begin(), p->conv50l.end());
      p->mgQH.conv50.assign(p->conv50l.begin(), p->conv50l.end());
    }
    p->mgQ.sconv = p->sconv[0];
    p->mgQH.sconv = p->sconv[1];
    p->mgQ.sconv_n = p->mgQH.sconv_n = p->sconv_n;
    plan_mg_buffers(p->mgQ, cv, p->csize);
    plan_mg_buffers(p->mgQH, cv, p->csize);
  } else {
    plan_mg_buffers(p->mgW, cv, p->csize);
  }
  plan_mg_buffers(p->mgK, cv, p->csize);
  const int m = p->o.restart;
  const bool freq = p->o.outer == PINTOC_OUTER_FGMRES_FREQ;
  for (Member& mb : p->mem) {
    const size_t vb = sizeof(double) * (size_t)std::max<int64_t>(mb.n_all, freq ? p->nF : 0);
    mb.Vk = cv.take<double>(vb * (m + 1));
    if (p->o.z_fp32)
      mb.Zk32 = cv.take<float>(vb / 2 * m);
    else
      mb.Zk = cv.take<double>(vb * m);
    mb.rvec = cv.take<double>(vb);
    mb.xtmp = cv.take<double>(vb);
  }
  p->Vk = p->mem[0].Vk;
  p->Zk = p->mem[0].Zk;
  p->rvec = p->mem[0].rvec;
  p->xtmp = p->mem[0].xtmp;
  p->dscale = p->side != 1.0 ? cv.take<double>(sizeof(double) * (size_t)p->n_all) : nullptr;
  if (freq) {
    p->fb = cv.take<double>(sizeof(double) * (size_t)p->nF);
    p->fsc = cv.take<double>(sizeof(double) * nf);
    p->fisc = cv.take<double>(sizeof(double) * nf);
    p->ftmp = cv.take<double>(sizeof(double) * 8 * (size_t)p->nq2);
    p->gcoef = cv.take<BlockCoef>(sizeof(BlockCoef) * nf);
  }
  p->dd = cv.take<double>(sizeof(double) * 64);
  p->dd2 = cv.take<double>(sizeof(double) * 64);
  p->part = cv.take<double>(sizeof(double) * 8 * 1024);
  p->need = cv.off;
}

// ------------------------------------------------------------ convection
// Element-by-element assembly (3x3 Gauss per element) of the convection
// matrices N[i][j] = int (w . grad phi_j) phi_i (Q2) and the same with the Q1
// basis, w the Q2 nodal interpolant of the wind, stored as node-centred
// stencil tables: Q2 50 values per node (25 offsets of N, 25 of N^T), Q1 18.
static void p2_1d(double s, double v[3], double d[3]) {
  v[0] = (1 - s) * (1 - 2 * s); v[1] = 4 * s * (1 - s); v[2] = s * (2 * s - 1);
  d[0] = 4 * s - 3; d[1] = 4 - 8 * s; d[2] = 4 * s - 1;
}

static void conv_tables(int n, const double* wx, const double* wy, std::vector<double>& t2, std::vector<double>* t1) {
  const int nq = 2 * n + 1, np = n + 1;
  const double h = 1.0 / n;
  const double g[3] = {0.5 - std::sqrt(15.0) / 10.0, 0.5, 0.5 + std::sqrt(15.0) / 10.0};
  const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  t2.assign((size_t)nq * nq * 50, 0.0);
  if (t1) t1->assign((size_t)np * np * 18, 0.0);
  for (int ey = 0; ey < n; ++ey)
    for (int ex = 0; ex < n; ++ex) {
      double Ne[9][9] = {}, Np[4][4] = {};
      for (int qy = 0; qy < 3; ++qy)
        for (int qx = 0; qx < 3; ++qx) {
          double vx[3], dx[3], vy[3], dy[3];
          p2_1d(g[qx], vx, dx);
          p2_1d(g[qy], vy, dy);
          const double lx[2] = {1 - g[qx], g[qx]}, ly[2] = {1 - g[qy], g[qy]};
          double phi[9], phx[9], phy[9];
          double wxq = 0, wyq = 0;
          for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
              const int l = 3 * b + a;
              phi[l] = vx[a] * vy[b];
              phx[l] = dx[a] / h * vy[b];
              phy[l] = vx[a] * dy[b] / h;
              const int node = (2 * ey + b) * nq + 2 * ex + a;
              wxq += wx[node] * phi[l];
              wyq += wy[node] * phi[l];
            }
          const double wt = gw[qx] * gw[qy] * h * h;
          for (int a = 0; a < 9; ++a)
            for (int b = 0; b < 9; ++b) Ne[a][b] += wt * phi[a] * (wxq * phx[b] + wyq * phy[b]);
          if (t1) {
            double psi[4], psx[4], psy[4];
            for (int b = 0; b < 2; ++b)
              for (int a = 0; a < 2; ++a) {
                const int l = 2 * b + a;
                psi[l] = lx[a] * ly[b];
                psx[l] = (a ? 1.0 : -1.0) / h * ly[b];
                psy[l] = lx[a] * (b ? 1.0 : -1.0) / h;
              }
            for (int a = 0; a < 4; ++a)
              for (int b = 0; b < 4; ++b) Np[a][b] += wt * psi[a] * (wxq * psx[b] + wyq * psy[b]);
          }
        }
      for (int a = 0; a < 9; ++a)
        for (int b = 0; b < 9; ++b) {
          const int ix = 2 * ex + a % 3, iy = 2 * ey + a / 3, jx = 2 * ex + b % 3, jy = 2 * ey + b / 3;
          const int ox = jx - ix, oy = jy - iy;
          t2[(size_t)(iy * nq + ix) * 50 + (oy + 2) * 5 + ox + 2] += Ne[a][b];
          t2[(size_t)(jy * nq + jx) * 50 + 25 + (-oy + 2) * 5 + (-ox + 2)] += Ne[a][b];
        }
      if (t1)
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) {
            const int ix = ex + a % 2, iy = ey + a / 2, jx = ex + b % 2, jy = ey + b / 2;
            const int ox = jx - ix, oy = jy - iy;
            (*t1)[(size_t)(iy * np + ix) * 18 + (oy + 1) * 3 + ox + 1] += Np[a][b];
            (*t1)[(size_t)(jy * np + jx) * 18 + 9 + (-oy + 1) * 3 + (-ox + 1)] += Np[a][b];
          }
    }
}

// ------------------------------------------------------------ public: options
extern "C" int pintoc_default_options(pintoc_options* o) {
  if (!o) return fail(PINTOC_EINVAL, "options pointer is NULL");
  o->inner = PINTOC_INNER_LINEAR;
  o->precision = PINTOC_PREC_FP64;
  o->restart = 10;
  o->max_outer = 200;
  o->tol = 1e-8;
  o->inner_tol = 1e-2;
  o->inner_restart = 50;
  o->inner_maxit = 200;
  o->n_vcycles = 4;
  o->n_cheb = 10;
  o->n_uzawa = 6;
  o->mu_uzawa = 0.75;
  o->stall_guard = 1;
  o->outer = PINTOC_OUTER_FGMRES;
  o->smoother = PINTOC_SMOOTHER_TILED;
  o->pressure_stream = 0;
  o->graphs = 0;
  o->z_fp32 = 0;
  return PINTOC_OK;
}

extern "C" const char* pintoc_last_error(void) { return g_err.c_str(); }

extern "C" int64_t pintoc_vector_length(const pintoc_problem* p) { return p ? p->n_all : 0; }

extern "C" int pintoc_profile_enable(pintoc_problem* p, int32_t enable) {
  if (!p) return fail(PINTOC_EINVAL, "NULL handle");
  MGPlan& m = p->d.flow == PINTOC_OSEEN ? p->mgQ : p->mgW;
  if (enable) {
    if (p->probe.create() != PINTOC_OK || p->probe_post.create() != PINTOC_OK)
      return fail(PINTOC_EHIP, "hipEventCreate failed");
    p->probe.count = p->probe_post.count = 0;
    p->probe.on = p->probe_post.on = true;
    m.probe = &p->probe;
    m.probe_post = &p->probe_post;
  } else {
    p->probe.on = p->probe_post.on = false;
  }
  return PINTOC_OK;
}

// mean duration and algorithmic bytes of the recorded launches of one probe
static int probe_mean(Probe& pr, double& ms_avg, int64_t& n_out, double& bytes_avg) {
  const long n = std::min<long>(pr.count, Probe::kCap);
  ms_avg = bytes_avg = 0.0;
  n_out = n;
  if (n == 0) return PINTOC_OK;
  double sum = 0, bytes = 0;
  for (long i = 0; i < n; ++i) {
    HIPCHK(hipEventSynchronize(pr.e1[i]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, pr.e0[i], pr.e1[i]));
    sum += ms;
    bytes += pr.bytes[i];
  }
  ms_avg = sum / n;
  bytes_avg = bytes / n;
  return PINTOC_OK;
}

extern "C" int pintoc_profile_read(pintoc_problem* p, pintoc_kernel_timing* out) {
  if (!p || !out) return fail(PINTOC_EINVAL, "NULL handle or output");
  if (std::min<long>(p->probe.count, Probe::kCap) == 0) return fail(PINTOC_ESTATE, "no timed launches recorded");
  int rc = probe_mean(p->probe, out->avg_ms, out->launches, out->algorithmic_bytes);
  if (rc != PINTOC_OK) return rc;
  return probe_mean(p->probe_post, out->post_avg_ms, out->post_launches, out->post_algorithmic_bytes);
}

extern "C" int pintoc_last_inner_iterations(const pintoc_problem* p, int32_t* counts, int32_t n) {
  if (!p || !counts) return fail(PINTOC_EINVAL, "NULL handle or array");
  if (p->o.inner == PINTOC_INNER_LINEAR) {
    const int k = std::min(n, p->nf);
    for (int j = 0; j < k; ++j) counts[j] = 0;
    return k;
  }
  if (p->last_its.empty()) return fail(PINTOC_ESTATE, "no GMRES-mode application yet");
  const int k = std::min(n, (int32_t)p->last_its.size());
  for (int j = 0; j < k; ++j) counts[j] = p->last_its[j];
  return k;
}

static void byte_model(pintoc_problem* p);

// Validation and set-up of one problem or of a group of problems (members)
// that share N, the flow, the domain, the wind and the options; the kept
// frequencies of all members form one batch (member k owns the frequencies
// f0 .. f0 + nt_k/2 of it), every per-frequency table carries its member's
// tau, beta and nu.
static int create_impl(const pintoc_problem_desc* ds, int nm, const pintoc_options* o, pintoc_problem** out) {
  if (!ds || !out) return fail(PINTOC_EINVAL, "NULL descriptor or output pointer");
  if (nm < 1 || nm > 4096) return fail(PINTOC_EINVAL, "a group needs 1 to 4096 members");
  pintoc_options opt;
  pintoc_default_options(&opt);
  if (o) opt = *o;
  const pintoc_problem_desc* d = &ds[0];
  for (int k = 0; k < nm; ++k) {
    const pintoc_problem_desc* e = &ds[k];
    const std::string who = nm > 1 ? "member " + std::to_string(k) + ": " : std::string();
    if (e->N < 2 || !pow2(e->N) || e->N > 4096) return fail(PINTOC_EINVAL, who + "N must be a power of two in [2, 4096]");
    if (e->nt < 2 || !pow2(e->nt) || e->nt > 1024) return fail(PINTOC_EINVAL, who + "nt must be a power of two in [2, 1024]");
    if (!(e->T > 0) || !(e->nu > 0) || !(e->beta > 0)) return fail(PINTOC_EINVAL, who + "T, nu and beta must be > 0");
    if (e->flow != PINTOC_STOKES && e->flow != PINTOC_OSEEN) return fail(PINTOC_EINVAL, who + "unknown flow");
    if (e->flow == PINTOC_OSEEN && !e->wind) return fail(PINTOC_EINVAL, who + "Oseen flow needs a wind");
    if (k > 0) {
      if (e->N != d->N || e->flow != d->flow) return fail(PINTOC_EINVAL, who + "group members need the same N and flow");
      if (e->x0 != d->x0 || e->y0 != d->y0 || e->x1 != d->x1 || e->y1 != d->y1)
        return fail(PINTOC_EINVAL, who + "group members need the same domain");
      if (e->flow == PINTOC_OSEEN) {
        const size_t nw = 2 * (size_t)(2 * d->N + 1) * (2 * d->N + 1);
        if (std::memcmp(e->wind, d->wind, nw * sizeof(double)) != 0)
          return fail(PINTOC_EINVAL, who + "group members need the same wind");
      }
    }
  }
  const bool unit = d->x0 == 0.0 && d->y0 == 0.0 && d->x1 == 0.0 && d->y1 == 0.0;
  const double side = unit ? 1.0 : d->x1 - d->x0;
  if (!unit && (!(side > 0) || !std::isfinite(side) || std::fabs((d->y1 - d->y0) - side) > 1e-12 * side))
    return fail(PINTOC_EINVAL, "the domain must be a square [x0, x1] x [y0, y1] with x1 - x0 = y1 - y0 > 0");
  if (nm > 1 && side != 1.0) return fail(PINTOC_EINVAL, "groups are set up on the unit square only");
  if (opt.inner != PINTOC_INNER_LINEAR && opt.inner != PINTOC_INNER_GMRES && opt.inner != PINTOC_INNER_MINRES)
    return fail(PINTOC_EINVAL, "unknown inner mode");
  if (opt.inner == PINTOC_INNER_GMRES &&
      (opt.inner_restart < 1 || opt.inner_restart > 100 || opt.inner_maxit < 1 || !(opt.inner_tol > 0)))
    return fail(PINTOC_EINVAL, "invalid inner GMRES options");
  if (opt.inner == PINTOC_INNER_MINRES && (d->flow != PINTOC_STOKES || opt.inner_maxit < 1 || !(opt.inner_tol > 0)))
    return fail(PINTOC_EINVAL, "inner MINRES needs the Stokes flow, inner_maxit >= 1 and inner_tol > 0");
  if (opt.precision != PINTOC_PREC_FP64 && opt.precision != PINTOC_PREC_FP32_INNER)
    return fail(PINTOC_EINVAL, "unknown precision");
  if (opt.restart < 1 || opt.restart > 60 || opt.max_outer < 1 || !(opt.tol > 0) || opt.n_vcycles < 1 ||
      opt.n_cheb < 1 || (opt.stall_guard != 0 && opt.stall_guard != 1))
    return fail(PINTOC_EINVAL, "invalid solver options");
  if (opt.outer != PINTOC_OUTER_FGMRES && opt.outer != PINTOC_OUTER_MINRES && opt.outer != PINTOC_OUTER_FGMRES_FREQ)
    return fail(PINTOC_EINVAL, "unknown outer method");
  if (opt.outer == PINTOC_OUTER_FGMRES_FREQ &&
      (nm > 1 || side != 1.0 || (d->flow == PINTOC_OSEEN && opt.precision != PINTOC_PREC_FP64)))
    return fail(PINTOC_EINVAL, "the frequency-domain FGMRES needs a single problem on the unit square "
                               "(and FP64 for Oseen)");
  if (opt.smoother != PINTOC_SMOOTHER_TILED && opt.smoother != PINTOC_SMOOTHER_GLOBAL)
    return fail(PINTOC_EINVAL, "unknown smoother");
  if (opt.pressure_stream != 0 && opt.pressure_stream != 1) return fail(PINTOC_EINVAL, "pressure_stream must be 0 or 1");
  if (opt.graphs != 0 && opt.graphs != 1) return fail(PINTOC_EINVAL, "graphs must be 0 or 1");
  if (opt.z_fp32 != 0 &&
      (opt.z_fp32 != 1 || opt.precision != PINTOC_PREC_FP32_INNER || opt.outer != PINTOC_OUTER_FGMRES))
    return fail(PINTOC_EINVAL, "z_fp32 needs FP32 inner solves and the time-domain FGMRES");
  if (opt.outer == PINTOC_OUTER_MINRES &&
      (nm > 1 || d->flow != PINTOC_STOKES || opt.inner != PINTOC_INNER_LINEAR || opt.restart < 4))
    return fail(PINTOC_EINVAL, "MINRES needs a single Stokes problem, the linear preconditioner and restart >= 4");
  auto* p = new pintoc_problem();
  p->d = *d;
  p->d.wind = nullptr;
  p->o = opt;
  p->group = nm > 1;
  // A square of side l is the unit square's problem with viscosity nu / l^2
  // and wind w / l: M, K, B, N(w) scale as l^2, 1, l and l, so the physical
  // matrix is D_r A' D_c with A' the unit-square matrix of (nu / l^2, w / l),
  // D_r = l^2 on momentum rows and l on divergence rows, D_c = 1/l on
  // pressure columns.  Everything below is set up for A'; the entry points
  // apply D_r, D_c (see kkt and precond).
  p->side = side;
  p->d.nu = d->nu / (side * side);
  std::vector<double> wsc;
  if (d->flow == PINTOC_OSEEN) {
    const size_t nw = 2 * (size_t)(2 * d->N + 1) * (2 * d->N + 1);
    wsc.assign(d->wind, d->wind + nw);
    for (double& v : wsc) v /= side;
  }
  const int N = d->N;
  p->nq2 = (2 * N + 1) * (2 * N + 1);
  p->np2 = (N + 1) * (N + 1);
  p->L = 2 * p->nq2 + p->np2;
  p->csize = opt.precision == PINTOC_PREC_FP64 ? 16 : 8;
  p->segV = 4 * p->nq2;
  p->segP = 2 * p->np2;
  int f0 = 0, tw0 = 0;
  for (int k = 0; k < nm; ++k) {
    Member m;
    m.nt = ds[k].nt;
    m.nf = m.nt / 2 + 1;
    m.f0 = f0;
    m.tw0 = tw0;
    m.T = ds[k].T;
    m.tau = ds[k].T / m.nt;
    m.nu = ds[k].nu / (side * side);
    m.beta = ds[k].beta;
    m.n_all = (int64_t)2 * m.nt * p->L;
    f0 += m.nf;
    tw0 += m.nt / 2;
    // twiddles exp(-2 pi i k / nt) of this member's FFT length
    for (int q = 0; q < m.nt / 2; ++q) {
      const double a = -2.0 * M_PI * q / m.nt;
      p->tw_h.push_back(make_double2(std::cos(a), std::sin(a)));
    }
    p->mem.push_back(m);
  }
  p->nf = f0;
  p->tau = p->mem[0].tau;
  p->n_all = p->mem[0].n_all;
  const bool oseen = d->flow == PINTOC_OSEEN;
  int nl = 0;
  for (int n = N; n >= 2; n >>= 1) ++nl;
  if (oseen) {
    // wind on every level by injection of the finest nodal values
    const int nq = 2 * N + 1;
    std::vector<double> wx(wsc.begin(), wsc.begin() + (size_t)nq * nq), wy(wsc.begin() + (size_t)nq * nq, wsc.end());
    p->conv2_h.resize(nl);
    for (int l = 0; l < nl; ++l) {
      const int n = N >> l, nql = 2 * n + 1, st = 1 << l;
      std::vector<double> lx((size_t)nql * nql), ly((size_t)nql * nql);
      for (int iy = 0; iy < nql; ++iy)
        for (int ix = 0; ix < nql; ++ix) {
          lx[(size_t)iy * nql + ix] = wx[(size_t)(iy * st) * nq + ix * st];
          ly[(size_t)iy * nql + ix] = wy[(size_t)(iy * st) * nq + ix * st];
        }
      conv_tables(n, lx.data(), ly.data(), p->conv2_h[l], l == 0 ? &p->conv1_h : nullptr);
      if (l == 0) {
        const size_t nn = (size_t)nql * nql;
        p->conv50t_h.resize(50 * nn);
        for (size_t g = 0; g < nn; ++g)
          for (int e = 0; e < 50; ++e) p->conv50t_h[(size_t)e * nn + g] = p->conv2_h[0][g * 50 + e];
      }
      if (l + 1 < nl)
        for (int hf = 0; hf < 2; ++hf) {
          p->tconv_h[hf].emplace_back(q2_tile_conv_entries(n));
          q2_tile_conv_table(n, p->conv2_h[l].data(), hf, p->tconv_h[hf].back().data());
        }
    }
    int l0 = 0;                                   // the levels of the one-launch small V-cycle
    while ((N >> l0) > kQ2SmallN) ++l0;
    if (l0 + 1 < nl) {
      p->sconv_n = N >> l0;
      std::vector<const double*> tabs;
      for (int l = l0; l + 1 < nl; ++l) tabs.push_back(p->conv2_h[l].data());
      for (int hf = 0; hf < 2; ++hf) {
        p->sconv_h[hf].assign(q2_small_conv_entries(p->sconv_n), 0.0);
        q2_small_conv_table(p->sconv_n, tabs, hf, p->sconv_h[hf].data());
      }
    }
  }
  MGPlan& W = p->mgW;
  W.q2 = true; W.N = N; W.nb = 4 * p->nf; W.fpc = 4; W.ncoef = p->nf; W.fpj = 4;
  double wmax = 0.0;                             // largest nodal wind speed (coarse-level viscosity)
  if (oseen)
    for (size_t i = 0; i < (size_t)p->nq2; ++i) wmax = std::max(wmax, std::hypot(wsc[i], wsc[(size_t)p->nq2 + i]));
  std::vector<double> visc((size_t)nl * p->nf);
  for (const Member& mb : p->mem) {
    // per-frequency constants (section 3.1-3.2): d_j = 1 - exp(-2 pi i j/nt),
    // c2 = (1/beta + d_c^2/tau^2)^{-1/2},  c1 = d_r / sqrt(tau^2/beta + d_c^2)
    const double tau = mb.tau, beta = mb.beta, nu = mb.nu, sb = std::sqrt(beta);
    for (int j = 0; j < mb.nf; ++j) {
      const int jg = mb.f0 + j;
      const double th = 2.0 * M_PI * j / mb.nt;
      const double dr = 1.0 - std::cos(th), dc = std::sin(th);
      const cd dj(dr, dc), djc(dr, -dc);
      const double c2 = 1.0 / std::sqrt(1.0 / beta + dc * dc / (tau * tau));
      const double c1 = dr / std::sqrt(tau * tau / beta + dc * dc);
      p->tj_h.push_back(make_double2(dc, c2));
      p->ab_h.push_back(make_double2(1.0 + c1, nu * c2));
      p->cj_h.push_back(make_double2(c1, c2 * nu));          // X = c1 M + c2 L, L = nu K
      W.coef_h.push_back(mkcoef(1.0 + c1, nu * c2));        // W_j = (1 + c1) M + c2 nu K
      p->ftau_h.push_back(tau);
      p->finvtau_h.push_back(1.0 / tau);
      p->fbeta_h.push_back(beta);
      p->fnu_h.push_back(nu);
      BlockCoef bc{};
      auto c2d = [](cd v) { return make_double2(v.real(), v.imag()); };
      if (!oseen) {          // Z_j = [[M, X, 0, B^T], [X, -M, B^T, 0], [0, B, 0, 0], [B, 0, 0, 0]]
        bc.a11 = c2d(1.0); bc.a12 = c2d(c1); bc.b12 = c2d(c2 * nu); bc.e12 = c2d(0.0);
        bc.a21 = c2d(c1); bc.b21 = c2d(c2 * nu); bc.e21 = c2d(0.0); bc.a22 = c2d(-1.0); bc.s = 1.0;
      } else {               // G_j of eq. (SubBlockG)
        bc.a11 = c2d(tau); bc.a12 = c2d(djc); bc.b12 = c2d(tau * nu); bc.e12 = c2d(tau);
        bc.a21 = c2d(dj); bc.b21 = c2d(tau * nu); bc.e21 = c2d(tau); bc.a22 = c2d(-tau / beta); bc.s = tau;
        // Psi = d M + tau L, Psi^H = conj(d) M + tau L^T (L = nu K + N);
        // Q_j = Psi + tau/sqrt(beta) M, Q_j^H = Psi^H + tau/sqrt(beta) M
        p->cpsi_h.push_back(mkcoef(dj, tau * nu, tau, 0.0));
        p->cpsih_h.push_back(mkcoef(djc, tau * nu, tau, 0.0));     // eta: applied to the N^T table
        p->mgQ.coef_h.push_back(mkcoef(dj + tau / sb, tau * nu, tau, 0.0));
        p->mgQH.coef_h.push_back(mkcoef(djc + tau / sb, tau * nu, 0.0, tau));
        p->dj_h.push_back(make_double2(dr, dc));
        // the mass operators of the Uzawa steps: tau M, tau/beta M, M
        p->cscal_h[0].push_back(mkcoef(tau, 0.0));
        p->cscal_h[1].push_back(mkcoef(tau / beta, 0.0));
        p->cscal_h[2].push_back(mkcoef(1.0, 0.0));
        p->abO_h.push_back(make_double2(-1.0 / (tau * tau), 0.0));
        // Coarse-level viscosity of the convection-diffusion multigrid: level
        // l of n x n elements (side h = 1/n) diffuses with tau max(nu,
        // |w|_max h / 4), so its mesh Peclet number |w|_max h / (2 nu_l) is at
        // most 2; the finest level keeps tau nu.  With the true nu on
        // convection-dominated coarse levels the V-cycle diverges.
        for (int l = 0; l < nl; ++l)
          visc[(size_t)l * p->nf + jg] = tau * (l == 0 ? nu : std::max(nu, wmax / (4.0 * (N >> l))));
      }
      p->bc_h.push_back(bc);
    }
  }
  MGPlan& K = p->mgK;
  K.q2 = false; K.N = N; K.nb = 2 * p->nf; K.fpc = 2 * p->nf; K.ncoef = 1; K.fpj = 2;
  K.coef_h.push_back(mkcoef(0.0, 1.0));                   // unconstrained pressure Laplacian
  for (MGPlan* m : {&p->mgQ, &p->mgQH}) {
    m->q2 = true; m->N = N; m->nb = 2 * p->nf; m->fpc = 2; m->ncoef = p->nf; m->fpj = 2;
  }
  if (oseen) {
    p->mgQ.visc = visc;
    p->mgQH.visc = visc;
  }
  std::vector<MGPlan*> plans = {&K};
  if (oseen) { plans.push_back(&p->mgQ); plans.push_back(&p->mgQH); }
  else plans.push_back(&W);
  for (MGPlan* m : plans) {
    m->nlev = nl;
    m->conv.assign(nl, nullptr);
    m->active = m->nb;
    for (int l = 0; l < nl; ++l)
      for (int set = 0; set < m->ncoef; ++set) {  // the Q2 tile kernels take the one nonzero half as eta
        OpCoef c = m->level_coef(set, l);
        if (m->q2 && (c.etat.x != 0.0 || c.etat.y != 0.0)) {
          if (c.eta.x != 0.0 || c.eta.y != 0.0) { delete p; return fail(PINTOC_EINVAL, "operator with N and N^T"); }
          c.eta = c.etat;
          c.etat = make_double2(0, 0);
        }
        m->coef_dev_h.push_back(c);
      }
    if (opt.smoother == PINTOC_SMOOTHER_GLOBAL) {
      m->global = true;
      for (int l = 0; l < nl; ++l)
        for (int set = 0; set < m->ncoef; ++set) m->coefg_h.push_back(m->level_coef(set, l));
    }
    const std::vector<double>* cc = (oseen && m->q2) ? &p->conv2_h[nl - 1] : nullptr;
    for (int set = 0; set < m->ncoef; ++set)
      if (!coarse_inverse(m->q2, m->level_coef(set, nl - 1), cc, m->inv_h)) {
        delete p;
        return fail(PINTOC_EINVAL, "singular coarse operator");
      }
  }
  p->mem_on.assign(nm, 1);
  p->freq_on.assign(p->nf, 1);
  if (opt.outer == PINTOC_OUTER_FGMRES_FREQ) {
    const Member& mb = p->mem[0];
    p->nF = (int64_t)2 * p->nf * (p->segV + p->segP);
    for (int j = 0; j < p->nf; ++j) {
      const double w = (j == 0 || 2 * j == mb.nt) ? 1.0 : 2.0;
      p->fsc_h.push_back(std::sqrt(w / mb.nt));
      p->fisc_h.push_back(1.0 / std::sqrt(w / mb.nt));
      // G_j of eq. (SubBlockG) for Stokes (no convection): the pattern of
      // oseen_kernels.hip with a11 = tau, a12 = conj(d), b = tau nu, a22 = -tau/beta, s = tau
      const double th = 2.0 * M_PI * j / mb.nt;
      BlockCoef g{};
      g.a11 = make_double2(mb.tau, 0.0);
      g.a12 = make_double2(1.0 - std::cos(th), -std::sin(th));
      g.b12 = make_double2(mb.tau * mb.nu, 0.0);
      g.a21 = make_double2(1.0 - std::cos(th), std::sin(th));
      g.b21 = make_double2(mb.tau * mb.nu, 0.0);
      g.a22 = make_double2(-mb.tau / mb.beta, 0.0);
      g.s = mb.tau;
      p->gc_h.push_back(g);
    }
  }
  carve(p, nullptr);
  byte_model(p);
  *out = p;
  return PINTOC_OK;
}

extern "C" int pintoc_problem_create(const pintoc_problem_desc* d, const pintoc_options* o, pintoc_problem** out) {
  return create_impl(d, 1, o, out);
}

extern "C" int pintoc_group_create(const pintoc_problem_desc* d, int32_t n, const pintoc_options* o,
                                   pintoc_problem** out) {
  if (n < 1) return fail(PINTOC_EINVAL, "a group needs at least one member");
  return create_impl(d, n, o, out);
}

extern "C" size_t pintoc_workspace_bytes(const pintoc_problem* p) { return p ? p->need : 0; }

// ------------------------------------------------------------ static scratch
// Device memory of the library itself, for callers that cannot allocate
// (pintoc_bind_scratch).  Each device the library runs on holds one copy of
// the array until the process ends.  In host code the array's name is no
// device address: its address on the current device comes from
// hipGetSymbolAddress, taken once per device and kept in g_scratch_ptr.  At
// most one problem per device is bound to it (g_scratch_owner); binding
// another problem takes the array over and unbinds the earlier one.
static constexpr size_t kScratchBytes = (size_t)128 << 20;
static constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices] = {};
static pintoc_problem* g_scratch_owner[kScratchDevices] = {};

// gives up p's hold on its device's scratch array (no-op if it has none)
static void scratch_release(pintoc_problem* p) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (p->scratch_dev >= 0 && g_scratch_owner[p->scratch_dev] == p) g_scratch_owner[p->scratch_dev] = nullptr;
  p->scratch_dev = -1;
}

extern "C" void pintoc_problem_destroy(pintoc_problem* p) {
  if (!p) return;
  scratch_release(p);
  if (p->pstream) {
    (void)hipStreamSynchronize(p->pstream);
    (void)hipStreamDestroy(p->pstream);
  }
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  for (GraphEntry& e : p->graphs) (void)hipGraphExecDestroy(e.exec);
  delete p;
}

static int bind_impl(pintoc_problem* p, void* dev, size_t bytes, hipStream_t s);

extern "C" int pintoc_bind_workspace(pintoc_problem* p, void* dev, size_t bytes, void* stream) {
  if (!p || !dev) return fail(PINTOC_EINVAL, "NULL handle or workspace");
  if (((uintptr_t)dev) & 255) return fail(PINTOC_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < p->need) return fail(PINTOC_ENOMEM, "workspace too small: need " + std::to_string(p->need) + " bytes");
  scratch_release(p);
  return bind_impl(p, dev, bytes, (hipStream_t)stream);
}

extern "C" int pintoc_bind_scratch(pintoc_problem* p, void* stream) {
  if (!p) return fail(PINTOC_EINVAL, "NULL handle");
  if (p->need > kScratchBytes)
    return fail(PINTOC_ENOMEM, "problem needs " + std::to_string(p->need) + " bytes of workspace, more than the " +
                                   std::to_string(kScratchBytes) + " bytes of the static scratch");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(PINTOC_EINVAL, "device index out of range");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* a = nullptr;
      const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !a)
        return fail(PINTOC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_scratch_ptr[dev] = a;
    }
    ptr = g_scratch_ptr[dev];
    pintoc_problem* prev = g_scratch_owner[dev];
    if (prev && prev != p) {              // the earlier problem loses its device memory
      prev->bound = false;
      prev->ws = nullptr;
      prev->scratch_dev = -1;
    }
    if (p->scratch_dev >= 0 && p->scratch_dev != dev && g_scratch_owner[p->scratch_dev] == p)
      g_scratch_owner[p->scratch_dev] = nullptr;
    g_scratch_owner[dev] = p;
    p->scratch_dev = dev;
  }
  return bind_impl(p, ptr, kScratchBytes, (hipStream_t)stream);
}

// carve the workspace, clear it and upload the tables on stream s
static int bind_impl(pintoc_problem* p, void* dev, size_t bytes, hipStream_t s) {
  p->bound = false;
  for (GraphEntry& e : p->graphs) (void)hipGraphExecDestroy(e.exec);   // captured with the old buffers
  p->graphs.clear();
  if (p->d.flow == PINTOC_STOKES && p->o.pressure_stream && !p->pstream) {
    HIPCHK(hipStreamCreateWithFlags(&p->pstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  }
  p->ws = dev;
  p->ws_bytes = bytes;
  carve(p, (char*)dev);
  // zero every buffer once: padded boundaries of all grids stay zero afterwards
  launch_fill_zero(s, (char*)dev, (p->need + 15) & ~(size_t)15);
  HIPCHK(hipMemcpyAsync(p->tw, p->tw_h.data(), sizeof(double2) * p->tw_h.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->ftau, p->ftau_h.data(), sizeof(double) * p->nf, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->finvtau, p->finvtau_h.data(), sizeof(double) * p->nf, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->fbeta, p->fbeta_h.data(), sizeof(double) * p->nf, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->fnu, p->fnu_h.data(), sizeof(double) * p->nf, hipMemcpyHostToDevice, s));
  if (p->fsc) {
    HIPCHK(hipMemcpyAsync(p->fsc, p->fsc_h.data(), sizeof(double) * p->nf, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->fisc, p->fisc_h.data(), sizeof(double) * p->nf, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->gcoef, p->gc_h.data(), sizeof(BlockCoef) * p->nf, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipMemcpyAsync(p->tj, p->tj_h.data(), sizeof(double2) * p->tj_h.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->ab, p->ab_h.data(), sizeof(double2) * p->ab_h.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->cj, p->cj_h.data(), sizeof(double2) * p->cj_h.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p->bc, p->bc_h.data(), sizeof(BlockCoef) * p->bc_h.size(), hipMemcpyHostToDevice, s));
  for (MGPlan* m : {&p->mgW, &p->mgK, &p->mgQ, &p->mgQH}) {
    if (m->nlev == 0 || !m->coef) continue;
    HIPCHK(hipMemcpyAsync(m->coef, m->coef_dev_h.data(), sizeof(OpCoef) * m->coef_dev_h.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(m->inv, m->inv_h.data(), sizeof(double2) * m->inv_h.size(), hipMemcpyHostToDevice, s));
    if (m->coefg)
      HIPCHK(hipMemcpyAsync(m->coefg, m->coefg_h.data(), sizeof(OpCoef) * m->coefg_h.size(), hipMemcpyHostToDevice, s));
  }
  if (p->d.flow == PINTOC_OSEEN) {
    HIPCHK(hipMemcpyAsync(p->conv50, p->conv2_h[0].data(), sizeof(double) * p->conv2_h[0].size(),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->conv50t, p->conv50t_h.data(), sizeof(double) * p->conv50t_h.size(),
                          hipMemcpyHostToDevice, s));
    auto upload = [&](void* dst, const std::vector<double>& t) -> int {
      if (p->csize == 16) {
        HIPCHK(hipMemcpyAsync(dst, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice, s));
      } else {                            // FP32 inner solves read FP32 tables
        const std::vector<float> f(t.begin(), t.end());
        HIPCHK(hipMemcpyAsync(dst, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));   // f is a temporary
      }
      return PINTOC_OK;
    };
    for (int hf = 0; hf < 2; ++hf) {
      for (size_t l = 0; l < p->tconv[hf].size(); ++l) {
        const int rc = upload(p->tconv[hf][l], p->tconv_h[hf][l]);
        if (rc != PINTOC_OK) return rc;
      }
      if (p->sconv[hf]) {
        const int rc = upload(p->sconv[hf], p->sconv_h[hf]);
        if (rc != PINTOC_OK) return rc;
      }
    }
    HIPCHK(hipMemcpyAsync(p->conv1, p->conv1_h.data(), sizeof(double) * p->conv1_h.size(), hipMemcpyHostToDevice, s));
    for (size_t l = 1; l < p->conv50l.size(); ++l)
      HIPCHK(hipMemcpyAsync(p->conv50l[l], p->conv2_h[l].data(), sizeof(double) * p->conv2_h[l].size(),
                            hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->cpsi, p->cpsi_h.data(), sizeof(OpCoef) * p->cpsi_h.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->cpsih, p->cpsih_h.data(), sizeof(OpCoef) * p->cpsih_h.size(), hipMemcpyHostToDevice, s));
    for (int q = 0; q < 3; ++q)
      HIPCHK(hipMemcpyAsync(p->cscal + (size_t)q * p->nf, p->cscal_h[q].data(), sizeof(OpCoef) * p->nf,
                            hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->dj, p->dj_h.data(), sizeof(double2) * p->dj_h.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->abO, p->abO_h.data(), sizeof(double2) * p->nf, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  p->bound = true;
  return PINTOC_OK;
}

// ------------------------------------------------------------ solve statistics
// Phase timing: an event pair around each phase of a solve (only while a
// solve runs).  Returns the slot to close, or -1.
static int phase_open(pintoc_problem* p, hipStream_t s, int phase) {
  auto& t = p->pt;
  if (!t.on) return -1;
  if (t.used == t.e0.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return -1; }
    t.e0.push_back(a); t.e1.push_back(b); t.phase.push_back(0);
  }
  const int k = (int)t.used++;
  t.phase[k] = phase;
  (void)hipEventRecord(t.e0[k], s);
  return k;
}
static void phase_close(pintoc_problem* p, hipStream_t s, int k) {
  if (k >= 0) (void)hipEventRecord(p->pt.e1[k], s);
}
// sums the recorded phases (waits for their events)
static void phase_sum(pintoc_problem* p, double out[PINTOC_NPHASES]) {
  for (int i = 0; i < PINTOC_NPHASES; ++i) out[i] = 0.0;
  auto& t = p->pt;
  for (size_t k = 0; k < t.used; ++k) {
    float ms = 0.0f;
    if (hipEventSynchronize(t.e1[k]) == hipSuccess && hipEventElapsedTime(&ms, t.e0[k], t.e1[k]) == hipSuccess)
      out[t.phase[k]] += 1e-3 * ms;
  }
}

// Byte model: compulsory HBM traffic of the passes as implemented (each
// field a kernel touches is read or written once; stencil tables, coefficient
// sets and the coarsest grids are left out).  Sizes: V = the four velocity
// grids of all kept frequencies, P = the two pressure grids, in the inner
// precision; C = one canonical FP64 vector.  A multigrid solve of c cycles
// costs (8.5 c - 1) passes per level on Q2 levels (pre-smoothing 3, 2 in the
// first cycle; fused residual/restriction 2.25; post-smoothing with the
// coarse correction 3.25) and (10.5 c - 1) on Q1 levels (residual 3 and
// restriction 1.25 instead), times 4/3 for the hierarchy; c Chebyshev steps
// 4 c - 3 passes.
static void byte_model(pintoc_problem* p) {
  const double cs = (double)p->csize, nf = p->nf;
  const double V = 4.0 * nf * p->nq2 * cs, P = 2.0 * nf * p->np2 * cs, H = V / 2.0;
  double C = 0.0;                        // the canonical vectors of all members
  for (const Member& mb : p->mem) C += 8.0 * (double)mb.n_all;
  const int c = p->o.n_vcycles, k = p->o.n_cheb;
  const double mg2 = (8.5 * c - 1.0) * 4.0 / 3.0, mg1 = (10.5 * c - 1.0) * 4.0 / 3.0, ch = 4.0 * k - 3.0;
  double block;
  if (p->d.flow == PINTOC_STOKES) {
    // W_j on 4 velocity grids, K_N and M_N on 2 pressure grids, unpin copy and combine
    block = mg2 * V + mg1 * P + ch * P + 2 * P + 3 * P;
  } else {
    // one Uzawa step on the half-blocks H: four operator products (2 each),
    // three combinations (4, 3, 4) and a final one (3), Chebyshev on M, two
    // multigrid solves (Q_j, Q_j^H) and the mass product between them (2)
    const double step = 4 * 2 * H + (4 + 3 + 4 + 3) * H + ch * H + 2 * mg2 * H + 2 * H;
    block = p->o.n_uzawa * step + 4 * H + 2 * H + 4 * H     // copies in, zero fill, copies out
            + (2 * P + 2 * H) + 2 * P + ch * P + 2 * P + 2 * P + mg1 * P + 2 * P;   // Schur step
  }
  p->model_fft = 2.0 * (C + V + P);
  p->model_block = block;                // all kept frequencies
  p->model_bmat = 2.0 * (V + P);         // block product Z_j / G_j, all frequencies
  p->model_fvec = V + P;                 // one frequency vector
  p->model_canon = C;
}

// ------------------------------------------------------------ multigrid
// One V(1,1)-cycle on level l: pre-smoothing x -> t (from x = 0 when x_zero,
// without reading x), residual and restriction (one fused pass on Q2 levels),
// coarse cycle from zero, and the
// post-smoothing sweep of t + P e_c -> x (the prolongation is applied while
// the sweep loads its tile).
template <typename R>
static void vcycle(hipStream_t s, MGPlan& m, int l, cpx<R>* x, const cpx<R>* b, bool x_zero) {
  const int n = m.n(l);
  const double h = 1.0 / n;
  if (l == m.nlev - 1) {
    launch_coarse<R>(s, m.q2, x, b, m.inv, m.fpc, m.nb, m.mk());
    return;
  }
  // every remaining level in one work-group per grid (Q2 convection from the
  // small-level table, which starts at level sconv_n)
  const bool small = m.q2 ? n <= kQ2SmallN && (!m.conv[l] || (m.sconv && n == m.sconv_n)) : !m.conv[l] && n <= kQ1SmallN;
  if (small) {
    if (m.q2)
      launch_q2_small_vcycle<R>(s, x, x_zero ? nullptr : x, b, n, m.coefl(l), m.ncoef, m.fpc, m.inv,
                                m.conv[l] ? (const R*)m.sconv : nullptr, m.nb, m.mk());
    else launch_q1_small_vcycle<R>(s, x, x_zero ? nullptr : x, b, n, m.coefl(l), m.fpc, m.inv, m.nb, m.mk());
    return;
  }
  cpx<R>* t = (cpx<R>*)m.t[l];
  cpx<R>* bc = (cpx<R>*)m.b[l + 1];
  cpx<R>* xc = (cpx<R>*)m.x[l + 1];
  if (m.global) {
    // multicolour Gauss-Seidel over whole grids: t = x (or 0), forward colour
    // sweep in place; after the coarse correction x = t + P e_c, backward sweep
    const size_t bytes = m.nodes(l) * m.nb * sizeof(cpx<R>);
    if (x_zero) launch_fill_zero(s, t, bytes);
    else (void)hipMemcpyAsync(t, x, bytes, hipMemcpyDeviceToDevice, s);
    const double* cv = m.conv50.empty() ? nullptr : m.conv50[l];
    launch_colour_sweep<R>(s, m.q2, t, b, n, h, m.coefgl(l), m.fpc, m.nb, cv, true, m.mk());
    cpx<R>* r = (cpx<R>*)m.r[l];
    if (m.q2) {
      launch_q2_residual_restrict<R>(s, bc, r, t, b, n, h, m.coefl(l), m.fpc, m.nb, (const R*)m.conv[l], m.mk());
    } else {
      launch_q1_residual<R>(s, r, t, b, n, h, m.coefl(l), m.fpc, m.nb, (const double*)m.conv[l], m.mk());
      launch_q1_restrict<R>(s, bc, r, n / 2, m.nb, m.mk());
    }
    vcycle<R>(s, m, l + 1, xc, bc, true);
    launch_prolong_add<R>(s, m.q2, x, t, xc, n, m.nb, m.mk());
    launch_colour_sweep<R>(s, m.q2, x, b, n, h, m.coefgl(l), m.fpc, m.nb, cv, false, m.mk());
    return;
  }
  // the probe times the finest pre-smoothing sweeps (reads b and, unless x = 0, x; writes t)
  Probe* pr = (l == 0 && m.probe && m.probe->on) ? m.probe : nullptr;
  const int slot = pr ? (int)(pr->count % Probe::kCap) : 0;
  if (pr) (void)hipEventRecord(pr->e0[slot], s);
  launch_tile_sweep<R>(s, m.q2, t, x_zero ? nullptr : x, b, nullptr, n, h, m.coefl(l), m.fpc, m.nb, m.conv[l], true,
                       m.mk());
  if (pr) {
    (void)hipEventRecord(pr->e1[slot], s);
    pr->bytes[slot] = (x_zero ? 2.0 : 3.0) * (double)m.nodes(0) * m.active * sizeof(cpx<R>);
    pr->count++;
  }
  cpx<R>* r = (cpx<R>*)m.r[l];
  if (m.q2) {
    launch_q2_residual_restrict<R>(s, bc, r, t, b, n, h, m.coefl(l), m.fpc, m.nb, (const R*)m.conv[l], m.mk());
  } else {
    launch_q1_residual<R>(s, r, t, b, n, h, m.coefl(l), m.fpc, m.nb, (const double*)m.conv[l], m.mk());
    launch_q1_restrict<R>(s, bc, r, n / 2, m.nb, m.mk());
  }
  vcycle<R>(s, m, l + 1, xc, bc, true);
  // the second probe times the finest post-smoothing sweeps (reads t, b and the
  // coarse correction, a quarter of a field; writes x)
  Probe* pp = (l == 0 && m.probe_post && m.probe_post->on) ? m.probe_post : nullptr;
  const int pslot = pp ? (int)(pp->count % Probe::kCap) : 0;
  if (pp) (void)hipEventRecord(pp->e0[pslot], s);
  launch_tile_sweep<R>(s, m.q2, x, t, b, xc, n, h, m.coefl(l), m.fpc, m.nb, m.conv[l], false, m.mk());
  if (pp) {
    (void)hipEventRecord(pp->e1[pslot], s);
    pp->bytes[pslot] = (3.0 * (double)m.nodes(0) + (double)m.nodes(1)) * m.active * sizeof(cpx<R>);
    pp->count++;
  }
}

// x = MG^cycles(b) from x = 0
template <typename R>
static void mg_solve(hipStream_t s, MGPlan& m, cpx<R>* x, const cpx<R>* b, int cycles) {
  for (int c = 0; c < cycles; ++c) vcycle<R>(s, m, 0, x, b, c == 0);
}

// Chebyshev semi-iteration (Jacobi-preconditioned, spectrum bounds [lo, hi] of
// diag(M)^{-1} M), ``steps`` steps from zero.  Returns the buffer holding x_steps.
template <typename R>
static cpx<R>* chebyshev(hipStream_t s, bool q2, int n, int nb, cpx<R>* A, cpx<R>* B, const cpx<R>* b, int steps,
                         double lo, double hi, Mask mk) {
  const double g = 2.0 / (lo + hi), sg = (hi - lo) / (hi + lo);
  const double h = 1.0 / n;
  launch_cheb<R>(s, q2, A, A, A, b, n, h, g, 1.0, 1, nb, mk);         // x_1 = g D^{-1} b
  cpx<R>*cur = A, *prev = B;
  double w = 1.0;
  for (int k = 1; k < steps; ++k) {
    w = k == 1 ? 1.0 / (1.0 - 0.5 * sg * sg) : 1.0 / (1.0 - 0.25 * sg * sg * w);
    // x_{k+1} overwrites x_{k-1}; the step from x_0 = 0 reads no x_{k-1}
    launch_cheb<R>(s, q2, prev, cur, k == 1 ? nullptr : prev, b, n, h, g, w, 0, nb, mk);
    std::swap(cur, prev);
  }
  return cur;
}

// ------------------------------------------------------------ preconditioner
// P~_j^{-1} (section 3.2) on a frequency vector: W_j^{-1} by V-cycles on the
// velocity fields, S^_j^{-1} = R L [(1+c1) K_N^+ + nu c2 M_N^{-1}] L^T R^T on
// the pressure fields.  in and out must not alias.
template <typename R>
// The pressure part (K_N multigrid, M_N Chebyshev) and the velocity part
// (W_j multigrid) touch disjoint buffers: with options.pressure_stream the
// pressure part runs on the problem's side stream, forked from s after the
// inputs and joined before the outputs are used, so its small latency-bound
// Q1 launches overlap the velocity V-cycles (the results do not depend on the
// overlap).
static void ptilde(pintoc_problem* p, hipStream_t s, const cpx<R>* inV, const cpx<R>* inP, cpx<R>* outV,
                   cpx<R>* outP) {
  const int nf = p->nf, cyc = p->o.n_vcycles, N = p->d.N;
  hipStream_t ps = s;
  if (p->pstream) {
    (void)hipEventRecord(p->ev_fork, s);
    (void)hipStreamWaitEvent(p->pstream, p->ev_fork, 0);
    ps = p->pstream;
  }
  cpx<R>* z = (cpx<R>*)p->Ptmp;
  launch_unpin_copy<R>(ps, z, inP, p->np2, 2 * nf, p->mk(2));
  mg_solve<R>(ps, p->mgK, (cpx<R>*)p->PxK, z, cyc);
  cpx<R>* ym = chebyshev<R>(ps, false, N, 2 * nf, (cpx<R>*)p->PxM, (cpx<R>*)p->PxM2, z, p->o.n_cheb, 0.25, 2.25,
                            p->mk(2));
  launch_schur_combine_pin<R>(ps, outP, (cpx<R>*)p->PxK, ym, p->ab, 2, p->np2, 2 * nf, p->mk(2));
  mg_solve<R>(s, p->mgW, outV, inV, cyc);
  if (p->pstream) {
    (void)hipEventRecord(p->ev_join, p->pstream);
    (void)hipStreamWaitEvent(s, p->ev_join, 0);
  }
}

// P~_j^(UZ)^{-1} of Algorithm 3 (Oseen) on a frequency vector, all kept
// frequencies at once.  (y1, y2) = k steps of eq. (Uzawa11) from zero on
// G_j^(1,1) with M^^{-1} = Chebyshev(M) and S^^{-1} = tau Q_j^{-H} M Q_j^{-1};
// (y3, y4) = -S^_j^{-1}((r3, r4) - tau (B y2, B y1)) with the commutator
// approximation carried onto the pinned pressure space.  in and out must not alias.
template <typename R>
static void puz(pintoc_problem* p, hipStream_t s, const cpx<R>* inV, const cpx<R>* inP, cpx<R>* outV,
                cpx<R>* outP) {
  const int nf = p->nf, N = p->d.N, cyc = p->o.n_vcycles;
  const double h = 1.0 / N;
  const size_t nh = (size_t)2 * nf * p->nq2;                  // complex entries of one velocity block
  cpx<R>*B1 = (cpx<R>*)p->B1, *B2 = (cpx<R>*)p->B2, *X1 = (cpx<R>*)p->X1, *X2 = (cpx<R>*)p->X2;
  cpx<R>*T1 = (cpx<R>*)p->T1, *T2 = (cpx<R>*)p->T2, *Rb = (cpx<R>*)p->Rb;
  const Mask m2 = p->mk(2);
  const int nq2 = p->nq2;
  launch_block_copy<R>(s, (cpx<R>*)inV, B1, N, nf, 0, 0, m2);
  launch_block_copy<R>(s, (cpx<R>*)inV, B2, N, nf, 1, 0, m2);
  launch_fill_zero(s, X1, nh * sizeof(cpx<R>));
  launch_fill_zero(s, X2, nh * sizeof(cpx<R>));
  const R *cvN = (const R*)p->tconv[0][0], *cvNT = (const R*)p->tconv[1][0];
  for (int k = 0; k < p->o.n_uzawa; ++k) {
    // x1 += tau^{-1} M^^{-1} (b1 - tau M x1 - Psi^H x2)
    launch_apply<R>(s, true, T1, X1, N, h, p->cscal + 0 * (size_t)nf, 2, 2 * nf, nullptr, m2);
    launch_apply<R>(s, true, T2, X2, N, h, p->cpsih, 2, 2 * nf, cvNT, m2);
    launch_combine3<R>(s, Rb, B1, T1, T2, 1.0, -1.0, -1.0, nullptr, nh, nq2, m2);
    cpx<R>* c = chebyshev<R>(s, true, N, 2 * nf, (cpx<R>*)p->C1, (cpx<R>*)p->C2, Rb, p->o.n_cheb, 0.25, 25.0 / 16.0,
                             m2);
    launch_combine3<R>(s, X1, X1, c, nullptr, 1.0, 1.0, 0.0, p->finvtau, nh, nq2, m2);   // 1/tau_j
    // x2 -= mu^{-1} S^^{-1} (b2 - Psi x1 + tau/beta M x2)
    launch_apply<R>(s, true, T1, X1, N, h, p->cpsi, 2, 2 * nf, cvN, m2);
    launch_apply<R>(s, true, T2, X2, N, h, p->cscal + 1 * (size_t)nf, 2, 2 * nf, nullptr, m2);
    launch_combine3<R>(s, Rb, B2, T1, T2, 1.0, -1.0, 1.0, nullptr, nh, nq2, m2);
    mg_solve<R>(s, p->mgQ, T1, Rb, cyc);                                   // Q_j^{-1}
    launch_apply<R>(s, true, T2, T1, N, h, p->cscal + 2 * (size_t)nf, 2, 2 * nf, nullptr, m2);   // M
    mg_solve<R>(s, p->mgQH, T1, T2, cyc);                                  // Q_j^{-H}
    launch_combine3<R>(s, X2, X2, T1, nullptr, 1.0, -1.0 / p->o.mu_uzawa, 0.0, p->ftau, nh, nq2, m2);
  }
  launch_block_copy<R>(s, outV, X1, N, nf, 0, 1, m2);
  launch_block_copy<R>(s, outV, X2, N, nf, 1, 1, m2);
  // Schur step on the pressure fields
  cpx<R>*Pt = (cpx<R>*)p->Pt, *Ub = (cpx<R>*)p->Ub, *z = (cpx<R>*)p->Ptmp;
  launch_schur_rhs<R>(s, Pt, inP, X1, X2, N, nf, p->ftau, m2);   // (r3 - tau B y2, r4 - tau B y1)
  launch_unpin_copy<R>(s, z, Pt, p->np2, 2 * nf, m2);
  cpx<R>* zz = chebyshev<R>(s, false, N, 2 * nf, (cpx<R>*)p->PxM, (cpx<R>*)p->PxM2, z, p->o.n_cheb, 0.25, 2.25, m2);
  launch_oseen_hp<R>(s, Ub, zz, N, nf, p->dj, p->ftau, p->fbeta, p->fnu, p->conv1, p->mk(1));
  launch_unpin_copy<R>(s, z, Ub, p->np2, 2 * nf, m2);
  mg_solve<R>(s, p->mgK, (cpx<R>*)p->PxK, z, cyc);
  launch_schur_combine_pin<R>(s, outP, (cpx<R>*)p->PxK, (cpx<R>*)p->PxK, p->abO, 2, p->np2, 2 * nf, m2);
}

// block preconditioner of the flow: P~_j (Stokes) or P~_j^(UZ) (Oseen)
template <typename R>
static void block_precond_eager(pintoc_problem* p, hipStream_t s, const cpx<R>* inV, const cpx<R>* inP,
                                cpx<R>* outV, cpx<R>* outP) {
  if (p->d.flow == PINTOC_OSEEN) puz<R>(p, s, inV, inP, outV, outP);
  else ptilde<R>(p, s, inV, inP, outV, outP);
}

// With options.graphs the launch sequence of one block preconditioner
// application (the V-cycles, Chebyshev and Uzawa steps of every frequency,
// 100-300 launches) is captured once per set of buffers and mask into a HIP
// graph and replayed: the kernels, their order and their arguments are the
// same, so the results equal the eager sequence bit for bit.  Eager instead
// while the kernel-timing probe records (its events are host bookkeeping), for
// the global smoother (its copies), or when s cannot capture (the legacy null
// stream); a capture that fails falls back to eager launches.
template <typename R>
static void block_precond(pintoc_problem* p, hipStream_t s, const cpx<R>* inV, const cpx<R>* inP, cpx<R>* outV,
                          cpx<R>* outP) {
  const bool probing = p->probe.on || p->probe_post.on;
  if (!p->o.graphs || probing || p->o.smoother == PINTOC_SMOOTHER_GLOBAL || s == nullptr) {
    block_precond_eager<R>(p, s, inV, inP, outV, outP);
    return;
  }
  const GraphKey key{inV, inP, outV, outP, p->cur_mask, (int)sizeof(R)};
  for (const GraphEntry& e : p->graphs)
    if (e.key == key) {
      if (hipGraphLaunch(e.exec, s) == hipSuccess) return;
      block_precond_eager<R>(p, s, inV, inP, outV, outP);
      return;
    }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone ||
      hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    block_precond_eager<R>(p, s, inV, inP, outV, outP);
    return;
  }
  block_precond_eager<R>(p, s, inV, inP, outV, outP);
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  const bool ok = hipStreamEndCapture(s, &g) == hipSuccess && g &&
                  hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!ok) {                                   // nothing ran: launch the sequence eagerly
    (void)hipGetLastError();
    block_precond_eager<R>(p, s, inV, inP, outV, outP);
    return;
  }
  p->graphs.push_back(GraphEntry{key, ex});
  if (hipGraphLaunch(ex, s) != hipSuccess) block_precond_eager<R>(p, s, inV, inP, outV, outP);
}

// block matrix of the flow: Z_j (Stokes) or G_j (Oseen)
template <typename R>
static void block_matvec(pintoc_problem* p, hipStream_t s, cpx<R>* yV, cpx<R>* yP, const cpx<R>* xV,
                         const cpx<R>* xP) {
  const bool oseen = p->d.flow == PINTOC_OSEEN;
  launch_block_mat<R>(s, yV, yP, xV, xP, p->d.N, p->nf, p->bc, oseen ? (const R*)p->tconv[0][0] : nullptr,
                      oseen ? (const R*)p->tconv[1][0] : nullptr, p->mk(2));
}

// Group members sitting out an application (converged ones): their
// frequencies are masked in every block kernel of the linear preconditioner.
static int member_mask(pintoc_problem* p, hipStream_t s) {
  bool all = true;
  for (int v : p->freq_on) all &= v != 0;
  if (all) return PINTOC_OK;
  p->mask_h = p->freq_on;
  HIPCHK(hipMemcpyAsync(p->maskd, p->mask_h.data(), sizeof(int) * p->nf, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  p->cur_mask = p->maskd;
  int on_count = 0;
  for (int v : p->freq_on) on_count += v != 0;
  for (MGPlan* m : {&p->mgW, &p->mgK, &p->mgQ, &p->mgQH}) { m->mask = p->maskd; m->active = on_count * m->fpj; }
  return PINTOC_OK;
}

static void clear_member_mask(pintoc_problem* p) {
  p->cur_mask = nullptr;
  for (MGPlan* m : {&p->mgW, &p->mgK, &p->mgQ, &p->mgQH}) { m->mask = nullptr; m->active = m->nb; }
}

// share of the batch's frequencies taking part (byte model)
static double active_fraction(const pintoc_problem* p) {
  int on = 0;
  for (int v : p->freq_on) on += v != 0;
  return p->nf ? (double)on / p->nf : 0.0;
}

// complex Givens rotation (c real) with [c, s; -conj(s), c] [a; b] = [r; 0]
static void givens(cd a, cd b, double& c, cd& sn) {
  if (b == 0.0) { c = 1.0; sn = 0.0; return; }
  if (a == 0.0) { c = 0.0; sn = std::conj(b) / std::abs(b); return; }
  const double t = std::hypot(std::abs(a), std::abs(b));
  c = std::abs(a) / t;
  sn = (a / std::abs(a)) * std::conj(b) / t;
}

// Batched right-preconditioned GMRES, one system Z_j x_j = s_j per kept
// frequency (Algorithm 2): x_0 = 0, restart m, stop for frequency j when the
// Arnoldi residual estimate satisfies |g_{k+1}| <= eps ||s_j||.  All
// frequencies advance in lockstep under a per-frequency mask.
//
// Orthogonalisation: classical Gram-Schmidt applied twice, with the second
// pass of column k - 1 carried out in the same sweep over the basis as the
// first pass of column k.  Iteration k holds final orthonormal q_0..q_{k-1}
// and the once-projected u_k (u_0 = q_0):
//   w^ = Z P~^{-1} u_k;  s = Q^H u_k, t = Q^H w^, nu = u_k^H u_k, mu = u_k^H w^
//   column k-1 += s,  H[k][k-1] = alpha = sqrt(nu - |s|^2),  q_k = (u_k - Q s)/alpha
//   since Z P~^{-1} q_k = (w^ - sum_i s_i Z P~^{-1} q_i)/alpha and
//   Z P~^{-1} q_i = sum_r H[r][i] q_r, with e = H[0:k+1, 0:k] s and
//   beta = (mu - s^H t)/alpha:
//     H[i][k] = (t_i - e_i)/alpha (i < k),  H[k][k] = (beta - e_k)/alpha,
//     u_{k+1} = (w^ - gamma u_k - Q (t - gamma s))/alpha,  gamma = beta/alpha.
// Column k is final once the next sweep adds Q_k^H u_{k+1}.  The stopping test
// is taken on final columns only: when the test on the tentative column k
// (subdiagonal ||u_{k+1}||) passes, a dot sweep finishes column k before the
// decision; a frequency whose final column k - 1 passes only at iteration k
// stops there (its last operator application is discarded).  Decisions and
// results equal those of Gram-Schmidt applied twice column by column.
template <typename R>
static int gmres_blocks(pintoc_problem* p, hipStream_t s) {
  const int nf = p->nf, m = p->o.inner_restart, segV = p->segV, segP = p->segP;
  const size_t ldV = (size_t)segV * nf, ldP = (size_t)segP * nf;
  cpx<R>*SV = (cpx<R>*)p->Vb, *SP = (cpx<R>*)p->Pb, *XV = (cpx<R>*)p->Vx, *XP = (cpx<R>*)p->Px;
  cpx<R>*BV = (cpx<R>*)p->BV, *BP = (cpx<R>*)p->BP, *ZV = (cpx<R>*)p->ZtV, *ZP = (cpx<R>*)p->ZtP;
  cpx<R>*UV = (cpx<R>*)p->UV, *UP = (cpx<R>*)p->UP;
  auto BVk = [&](int k) { return BV + (size_t)k * ldV; };
  auto BPk = [&](int k) { return BP + (size_t)k * ldP; };
  std::vector<double2> hb((size_t)(2 * m + 2) * nf), scl(nf), yv((size_t)(m + 1) * nf), rho(nf);
  std::vector<double2> csh((size_t)m * nf), cch((size_t)m * nf), agh((size_t)2 * nf);
  auto fetch = [&](double2* dev, std::vector<double2>& host, int k) -> int {
    HIPCHK(hipMemcpyAsync(host.data(), dev, sizeof(double2) * k * nf, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return PINTOC_OK;
  };
  auto upload = [&](double2* dev, const std::vector<double2>& host, int k) -> int {
    HIPCHK(hipMemcpyAsync(dev, host.data(), sizeof(double2) * k * nf, hipMemcpyHostToDevice, s));
    return PINTOC_OK;
  };
  int rc;
  // the mask in force for the block operations: frequencies still iterating
  auto set_mask = [&](const std::vector<int>& on) -> int {
    p->mask_h = on;
    HIPCHK(hipMemcpyAsync(p->maskd, p->mask_h.data(), sizeof(int) * nf, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    p->cur_mask = p->maskd;
    int on_count = 0;
    for (int v : on) on_count += v != 0;
    for (MGPlan* m : {&p->mgW, &p->mgK, &p->mgQ, &p->mgQH}) { m->mask = p->maskd; m->active = on_count * m->fpj; }
    return PINTOC_OK;
  };
  auto clear_mask = [&]() {
    p->cur_mask = nullptr;
    for (MGPlan* m : {&p->mgW, &p->mgK, &p->mgQ, &p->mgQH}) { m->mask = nullptr; m->active = m->nb; }
  };
  clear_mask();
  // ||s_j||
  launch_fdot<R>(s, SV, SP, 0, 0, 1, SV, SP, segV, segP, nf, p->fpart, p->hdev, kAll);
  if ((rc = fetch(p->hdev, hb, 1))) return rc;
  std::vector<double> bnorm(nf), rnorm(nf);
  std::vector<int> done(nf, 0), its(nf, 0), stalled(nf, 0);
  for (int j = 0; j < nf; ++j) {
    bnorm[j] = std::sqrt(std::max(hb[j].x, 0.0));
    rnorm[j] = bnorm[j];
    if (!(bnorm[j] > 0) || !p->freq_on[j]) done[j] = 1;     // nothing to solve, or a member sitting out
  }
  launch_fill_zero(s, XV, (size_t)segV * nf * sizeof(cpx<R>));
  launch_fill_zero(s, XP, (size_t)segP * nf * sizeof(cpx<R>));
  // per-frequency Hessenberg columns (unrotated), committed Givens rotations, g
  std::vector<cd> H((size_t)nf * (m + 1) * m), sn((size_t)nf * m), g((size_t)nf * (m + 1));
  std::vector<double> cs((size_t)nf * m);
  std::vector<char> fin((size_t)nf * m);
  auto Hj = [&](int j, int r, int c) -> cd& { return H[((size_t)j * (m + 1) + r) * m + c]; };
  std::vector<cd> col(m + 2);
  auto rotated = [&](int j, int k) {          // column k with rotations 0..k-1 applied
    for (int r = 0; r <= k + 1; ++r) col[r] = Hj(j, r, k);
    for (int i = 0; i < k; ++i) {
      const cd a = col[i], c = col[i + 1];
      const double ci = cs[(size_t)j * m + i];
      const cd si = sn[(size_t)j * m + i];
      col[i] = ci * a + si * c;
      col[i + 1] = -std::conj(si) * a + ci * c;
    }
  };
  auto commit = [&](int j, int k) -> double {  // rotation k of a final column; |g[k+1]|
    rotated(j, k);
    double ck; cd sk;
    givens(col[k], col[k + 1], ck, sk);
    cs[(size_t)j * m + k] = ck;
    sn[(size_t)j * m + k] = sk;
    cd* gj = g.data() + (size_t)j * (m + 1);
    gj[k + 1] = -std::conj(sk) * gj[k];
    gj[k] = ck * gj[k];
    return std::abs(gj[k + 1]);
  };
  auto tentative = [&](int j, int k) -> double {
    rotated(j, k);
    double ck; cd sk;
    givens(col[k], col[k + 1], ck, sk);
    return std::abs(std::conj(sk) * g[(size_t)j * (m + 1) + k]);
  };
  const cpx<R>*RV = SV, *RP = SP;          // residual of the current cycle
  int total = 0;
  while (true) {
    bool any = false;
    for (int j = 0; j < nf; ++j) any |= !done[j];
    if (!any || total >= p->o.inner_maxit) break;
    // q_0 = r / ||r|| for the frequencies still running
    std::vector<int> running(nf);
    for (int j = 0; j < nf; ++j) running[j] = !done[j];
    if ((rc = set_mask(running))) return rc;
    for (int j = 0; j < nf; ++j) scl[j] = make_double2(done[j] ? 0.0 : 1.0 / rnorm[j], 0.0);
    if ((rc = upload(p->ydev, scl, 1))) return rc;
    launch_fscale<R>(s, BVk(0), BPk(0), RV, RP, p->ydev, segV, segP, nf, p->mk(1));
    std::vector<int> kj(nf, 0), active = running;
    std::fill(H.begin(), H.end(), cd(0.0));
    std::fill(g.begin(), g.end(), cd(0.0));
    std::fill(fin.begin(), fin.end(), 0);
    for (int j = 0; j < nf; ++j) g[(size_t)j * (m + 1)] = rnorm[j];
    auto any_of = [&](const std::vector<int>& v) {
      for (int x : v) if (x) return true;
      return false;
    };
    int k = 0;
    for (; k < m; ++k) {
      if (active != p->mask_h && (rc = set_mask(active))) return rc;
      // operator on the once-projected u_k, then the fused dot sweep
      block_precond<R>(p, s, BVk(k), BPk(k), ZV, ZP);
      block_matvec<R>(p, s, BVk(k + 1), BPk(k + 1), ZV, ZP);
      launch_fdot_lag<R>(s, BV, BP, ldV, ldP, k, BVk(k), BPk(k), BVk(k + 1), BPk(k + 1), segV, segP, nf, p->fpart,
                         p->lagOut, p->mk(1));
      if ((rc = fetch(p->lagOut, hb, 2 * k + 2))) return rc;
      std::vector<int> upd = active;
      for (int j = 0; j < nf; ++j) {
        if (!active[j]) continue;
        auto sv = [&](int i) { const double2 v = hb[(size_t)i * nf + j]; return cd(v.x, v.y); };
        auto tv = [&](int i) { const double2 v = hb[(size_t)(k + i) * nf + j]; return cd(v.x, v.y); };
        const double nu = hb[(size_t)(2 * k) * nf + j].x;
        const cd mu(hb[(size_t)(2 * k + 1) * nf + j].x, hb[(size_t)(2 * k + 1) * nf + j].y);
        double alpha = 1.0;
        if (k > 0) {
          if (!fin[(size_t)j * m + k - 1]) {           // finish column k - 1
            double ss = 0;
            for (int i = 0; i < k; ++i) { Hj(j, i, k - 1) += sv(i); ss += std::norm(sv(i)); }
            Hj(j, k, k - 1) = std::sqrt(std::max(nu - ss, 0.0));
            fin[(size_t)j * m + k - 1] = 1;
            if (commit(j, k - 1) <= p->o.inner_tol * bnorm[j] || Hj(j, k, k - 1) == 0.0) {
              done[j] = 1; kj[j] = k; upd[j] = 0;
              continue;
            }
          }
          alpha = Hj(j, k, k - 1).real();
        }
        // first pass of column k from the sweep's dot products
        cd stt = 0.0;
        for (int i = 0; i < k; ++i) stt += std::conj(sv(i)) * tv(i);
        const cd bk = (mu - stt) / alpha, gam = bk / alpha;
        for (int r = 0; r <= k; ++r) {
          cd e = 0.0;
          for (int l = std::max(r - 1, 0); l < k; ++l) e += Hj(j, r, l) * sv(l);
          Hj(j, r, k) = (r < k ? tv(r) - e : bk - e) / alpha;
        }
        for (int i = 0; i < k; ++i) {
          const cd si = sv(i), ci = tv(i) - gam * si;
          csh[(size_t)i * nf + j] = make_double2(si.real(), si.imag());
          cch[(size_t)i * nf + j] = make_double2(ci.real(), ci.imag());
        }
        agh[j] = make_double2(alpha, 0.0);
        agh[nf + j] = make_double2(gam.real(), gam.imag());
      }
      active = upd;
      if (!any_of(active)) break;
      // fused update sweep: q_k, u_{k+1} and ||u_{k+1}||^2
      if (active != p->mask_h && (rc = set_mask(active))) return rc;
      if (k > 0 && ((rc = upload(p->lagCS, csh, k)) || (rc = upload(p->lagCC, cch, k)))) return rc;
      if ((rc = upload(p->lagAG, agh, 2))) return rc;
      launch_fupdate_lag<R>(s, BV, BP, ldV, ldP, k, p->lagCS, p->lagCC, p->lagAG, segV, segP, nf, p->fpart, p->lagRho,
                            p->mk(1));
      if ((rc = fetch(p->lagRho, rho, 1))) return rc;
      ++total;
      // tentative test on column k; finish it at once where it passes or the cycle ends
      std::vector<int> fnl(nf, 0);
      bool anyf = false;
      const bool last = k + 1 == m || total >= p->o.inner_maxit;
      for (int j = 0; j < nf; ++j) {
        if (!active[j]) continue;
        its[j]++;
        const double r2 = std::max(rho[j].x, 0.0);
        Hj(j, k + 1, k) = std::sqrt(r2);
        if (last || r2 == 0.0 || tentative(j, k) <= p->o.inner_tol * bnorm[j]) { fnl[j] = 1; anyf = true; }
      }
      if (anyf) {
        if ((rc = set_mask(fnl))) return rc;
        launch_fdot_lag<R>(s, BV, BP, ldV, ldP, k + 1, BVk(k + 1), BPk(k + 1), (const cpx<R>*)nullptr,
                           (const cpx<R>*)nullptr, segV, segP, nf, p->fpart, p->lagOut, p->mk(1));
        if ((rc = fetch(p->lagOut, hb, 2 * k + 4))) return rc;
        for (int j = 0; j < nf; ++j) {
          if (!fnl[j]) continue;
          double ss = 0;
          for (int i = 0; i <= k; ++i) {
            const cd si(hb[(size_t)i * nf + j].x, hb[(size_t)i * nf + j].y);
            Hj(j, i, k) += si;
            ss += std::norm(si);
          }
          Hj(j, k + 1, k) = std::sqrt(std::max(hb[(size_t)(2 * k + 2) * nf + j].x - ss, 0.0));
          fin[(size_t)j * m + k] = 1;
          const double res = commit(j, k);
          if (res <= p->o.inner_tol * bnorm[j] || Hj(j, k + 1, k) == 0.0) {
            done[j] = 1; kj[j] = k + 1; active[j] = 0;
          } else if (last) {
            kj[j] = k + 1; active[j] = 0;
            // stagnation guard: a whole restart cycle without halving the residual
            if (p->o.stall_guard && res > 0.5 * bnorm[j]) stalled[j] = 1;
          }
        }
      }
      if (!any_of(active)) { ++k; break; }
    }
    // y_j = R_j^{-1} g_j (size kj), U = sum_i y_ij q_i, X += P~^{-1} U
    std::fill(yv.begin(), yv.end(), make_double2(0, 0));
    int kmax = 0;
    for (int j = 0; j < nf; ++j) {
      if (!running[j]) continue;
      const int kk = kj[j];
      kmax = std::max(kmax, kk);
      std::vector<cd> Rm((size_t)kk * kk), y(kk);
      for (int c = 0; c < kk; ++c) {
        rotated(j, c);
        const double ck = cs[(size_t)j * m + c];
        const cd sk = sn[(size_t)j * m + c];
        col[c] = ck * col[c] + sk * col[c + 1];
        for (int r = 0; r <= c; ++r) Rm[(size_t)r * kk + c] = col[r];
      }
      const cd* gj = g.data() + (size_t)j * (m + 1);
      for (int i = kk - 1; i >= 0; --i) {
        cd v = gj[i];
        for (int q = i + 1; q < kk; ++q) v -= Rm[(size_t)i * kk + q] * y[q];
        y[i] = v / Rm[(size_t)i * kk + i];
      }
      for (int i = 0; i < kk; ++i) yv[(size_t)i * nf + j] = make_double2(y[i].real(), y[i].imag());
    }
    if ((rc = upload(p->ydev, yv, kmax))) return rc;
    if ((rc = set_mask(running))) return rc;                 // every frequency that ran in this cycle
    launch_fill_zero(s, UV, (size_t)segV * nf * sizeof(cpx<R>));
    launch_fill_zero(s, UP, (size_t)segP * nf * sizeof(cpx<R>));
    launch_fupdate<R>(s, UV, UP, BV, BP, ldV, ldP, kmax, p->ydev, segV, segP, nf, -1.0, p->mk(1));
    block_precond<R>(p, s, UV, UP, ZV, ZP);
    for (int j = 0; j < nf; ++j) scl[j] = make_double2(1.0, 0.0);
    if ((rc = upload(p->hdev, scl, 1))) return rc;
    launch_fupdate<R>(s, XV, XP, ZV, ZP, 0, 0, 1, p->hdev, segV, segP, nf, -1.0, p->mk(1));   // X += P~^{-1} U
    bool any_left = false;
    for (int j = 0; j < nf; ++j) {
      if (stalled[j]) done[j] = 1;                         // given up: keeps its approximate solution
      any_left |= !done[j];
    }
    if (!any_left || total >= p->o.inner_maxit) break;
    // restart: r = s - Z x for the frequencies still running
    for (int j = 0; j < nf; ++j) running[j] = !done[j];
    if ((rc = set_mask(running))) return rc;
    block_matvec<R>(p, s, UV, UP, XV, XP);
    for (int j = 0; j < nf; ++j) scl[j] = make_double2(-1.0, 0.0);
    if ((rc = upload(p->hdev, scl, 1))) return rc;
    launch_fscale<R>(s, UV, UP, UV, UP, p->hdev, segV, segP, nf, p->mk(1));
    for (int j = 0; j < nf; ++j) scl[j] = make_double2(1.0, 0.0);
    if ((rc = upload(p->h2dev, scl, 1))) return rc;
    launch_fupdate<R>(s, UV, UP, SV, SP, 0, 0, 1, p->h2dev, segV, segP, nf, -1.0, p->mk(1));   // U = s - Z x
    launch_fdot<R>(s, UV, UP, 0, 0, 1, UV, UP, segV, segP, nf, p->fpart, p->hdev, p->mk(1));
    if ((rc = fetch(p->hdev, hb, 1))) return rc;
    for (int j = 0; j < nf; ++j) rnorm[j] = std::sqrt(std::max(hb[j].x, 0.0));
    RV = UV; RP = UP;
  }
  clear_mask();
  p->last_its = its;
  if ((int)p->its_acc.size() != nf) p->its_acc.assign(nf, 0);
  {
    // model: per frequency, each iteration k applies the block preconditioner
    // and the block product and reads the basis twice (2 k + 6 vector passes);
    // each restart cycle ends with one more preconditioner application
    const double per_j_block = p->model_block / nf, per_j_bmat = p->model_bmat / nf, fv = p->model_fvec / nf;
    for (int j = 0; j < nf; ++j) {
      const double kk = its[j];
      const double cycles = its[j] > 0 ? std::ceil(kk / m) : 0.0;
      p->bytes_acc += (kk + cycles) * per_j_block + kk * per_j_bmat + (kk * (kk - 1.0) + 6.0 * kk) * fv;
    }
  }
  for (int j = 0; j < nf; ++j) {
    if (!p->freq_on[j]) continue;
    p->its_acc[j] += its[j];
    p->inner_its_sum += its[j];
    p->inner_blocks += 1;
    p->inner_its_max = std::max(p->inner_its_max, its[j]);
  }
  return PINTOC_OK;
}

// Batched preconditioned MINRES, one system Z_j x_j = s_j per kept frequency
// (the inner-solver variant of Algorithm 2 for Stokes: Z_j real symmetric,
// P~_j Hermitian positive definite on the complex frequency vectors).  All
// frequencies advance in lockstep under a per-frequency mask; the Lanczos
// and Givens scalars are real and kept on the host, one short recurrence per
// frequency (Paige and Saunders):
//   z = z^ / g,  delta = <z, Z z>,  v+ = Z z - (delta/g) v - (g/g-) v-,
//   z^+ = P~^{-1} v+,  g+ = sqrt(<v+, z^+>),
//   a0 = c delta - c- s g,  a1 = hypot(a0, g+),  a2 = s delta + c- c g,
//   a3 = s- g,  (c, s) <- (a0, g+) / a1,
//   w+ = (z - a3 w- - a2 w) / a1,  x += c eta w+,  eta <- -s eta,
// stopping when |eta| <= eps g_1 (eta is the P~_j-norm of the residual, g_1
// that of s_j).  The scaling by 1/g is folded into the update coefficients,
// so z^ is never rescaled in memory.  Block vectors: three Lanczos vectors,
// two preconditioned ones, two search directions (seven in all).
template <typename R>
static int minres_blocks(pintoc_problem* p, hipStream_t s) {
  const int nf = p->nf, segV = p->segV, segP = p->segP;
  const size_t ldV = (size_t)segV * nf, ldP = (size_t)segP * nf;
  cpx<R>*SV = (cpx<R>*)p->Vb, *SP = (cpx<R>*)p->Pb, *XV = (cpx<R>*)p->Vx, *XP = (cpx<R>*)p->Px;
  cpx<R>*BV = (cpx<R>*)p->BV, *BP = (cpx<R>*)p->BP;
  auto BVk = [&](int k) { return BV + (size_t)k * ldV; };
  auto BPk = [&](int k) { return BP + (size_t)k * ldP; };
  double* cf = (double*)p->ydev;                          // 3 nf update coefficients
  std::vector<double2> hb(nf), unit(nf, make_double2(1.0, 0.0));
  std::vector<double> cfh((size_t)3 * nf, 0.0);
  int rc;
  auto fetch = [&]() -> int {
    HIPCHK(hipMemcpyAsync(hb.data(), p->hdev, sizeof(double2) * nf, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return PINTOC_OK;
  };
  auto set_mask = [&](const std::vector<int>& on) -> int {
    p->mask_h = on;
    HIPCHK(hipMemcpyAsync(p->maskd, p->mask_h.data(), sizeof(int) * nf, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    p->cur_mask = p->maskd;
    int on_count = 0;
    for (int v : on) on_count += v != 0;
    for (MGPlan* m : {&p->mgW, &p->mgK, &p->mgQ, &p->mgQH}) { m->mask = p->maskd; m->active = on_count * m->fpj; }
    return PINTOC_OK;
  };
  auto comb = [&](int y, const cpx<R>* x1V, const cpx<R>* x1P, const cpx<R>* x2V, const cpx<R>* x2P) -> int {
    HIPCHK(hipMemcpyAsync(cf, cfh.data(), sizeof(double) * 3 * nf, hipMemcpyHostToDevice, s));
    cpx<R>* yV = y < 0 ? XV : BVk(y);
    cpx<R>* yP = y < 0 ? XP : BPk(y);
    launch_fcomb3<R>(s, yV, yP, x1V, x1P, x2V, x2P, cf, segV, segP, nf, p->mk(1));
    HIPCHK(hipStreamSynchronize(s));                       // cfh is rewritten by the next call
    return PINTOC_OK;
  };
  std::vector<int> done(nf, 0), its(nf, 0);
  for (int j = 0; j < nf; ++j) done[j] = !p->freq_on[j];
  // slots: Lanczos vectors v-, v, v+ and z^, z^+, search directions w-, w
  int iv0 = 0, iv = 1, iv1 = 2, iz = 3, iz1 = 4, iw0 = 5, iw = 6;
  for (int k : {iv0, iw0, iw}) {
    launch_fill_zero(s, BVk(k), ldV * sizeof(cpx<R>));
    launch_fill_zero(s, BPk(k), ldP * sizeof(cpx<R>));
  }
  launch_fill_zero(s, XV, ldV * sizeof(cpx<R>));
  launch_fill_zero(s, XP, ldP * sizeof(cpx<R>));
  std::vector<int> active(nf);
  for (int j = 0; j < nf; ++j) active[j] = !done[j];
  if ((rc = set_mask(active))) return rc;
  HIPCHK(hipMemcpyAsync(p->h2dev, unit.data(), sizeof(double2) * nf, hipMemcpyHostToDevice, s));
  launch_fscale<R>(s, BVk(iv), BPk(iv), SV, SP, p->h2dev, segV, segP, nf, p->mk(1));    // v = s_j
  block_precond<R>(p, s, BVk(iv), BPk(iv), BVk(iz), BPk(iz));
  launch_fdot<R>(s, BVk(iv), BPk(iv), 0, 0, 1, BVk(iz), BPk(iz), segV, segP, nf, p->fpart, p->hdev, p->mk(1));
  if ((rc = fetch())) return rc;
  std::vector<double> g(nf), g0(nf, 1.0), g1(nf), eta(nf), c(nf, 1.0), c0(nf, 1.0), sn(nf, 0.0), sn0(nf, 0.0),
      delta(nf), gn(nf), g2(nf);
  for (int j = 0; j < nf; ++j) {
    if (done[j]) continue;
    g[j] = std::sqrt(std::max(hb[j].x, 0.0));
    g1[j] = eta[j] = g[j];
    if (!(g[j] > 0)) done[j] = 1;
  }
  int total = 0;
  while (total < p->o.inner_maxit) {
    bool any = false;
    for (int j = 0; j < nf; ++j) any |= (active[j] = !done[j]) != 0;
    if (!any) break;
    if (active != p->mask_h && (rc = set_mask(active))) return rc;
    // Z z^ and <z^, Z z^>
    block_matvec<R>(p, s, BVk(iv1), BPk(iv1), BVk(iz), BPk(iz));
    launch_fdot<R>(s, BVk(iz), BPk(iz), 0, 0, 1, BVk(iv1), BPk(iv1), segV, segP, nf, p->fpart, p->hdev, p->mk(1));
    if ((rc = fetch())) return rc;
    for (int j = 0; j < nf; ++j) {
      if (!active[j]) continue;
      delta[j] = hb[j].x / (g[j] * g[j]);
      cfh[j] = 1.0 / g[j];                                  // v+ = (Z z^)/g - (delta/g) v - (g/g-) v-
      cfh[nf + j] = -delta[j] / g[j];
      cfh[2 * nf + j] = -g[j] / g0[j];
    }
    if ((rc = comb(iv1, BVk(iv), BPk(iv), BVk(iv0), BPk(iv0)))) return rc;
    block_precond<R>(p, s, BVk(iv1), BPk(iv1), BVk(iz1), BPk(iz1));
    launch_fdot<R>(s, BVk(iv1), BPk(iv1), 0, 0, 1, BVk(iz1), BPk(iz1), segV, segP, nf, p->fpart, p->hdev, p->mk(1));
    if ((rc = fetch())) return rc;
    std::vector<int> upd = active;
    std::vector<double> step(nf, 0.0);
    for (int j = 0; j < nf; ++j) {
      if (!active[j]) continue;
      g2[j] = hb[j].x;
      gn[j] = std::sqrt(std::max(g2[j], 0.0));
      const double a0 = c[j] * delta[j] - c0[j] * sn[j] * g[j];
      const double a1 = std::hypot(a0, gn[j]);
      const double a2 = sn[j] * delta[j] + c0[j] * c[j] * g[j];
      const double a3 = sn0[j] * g[j];
      if (!(a1 > 0)) {                                      // breakdown: keep the iterate
        done[j] = 1;
        upd[j] = 0;
        continue;
      }
      c0[j] = c[j];
      sn0[j] = sn[j];
      c[j] = a0 / a1;
      sn[j] = gn[j] / a1;
      cfh[j] = -a3 / a1;                                    // w+ (in the w- slot) = z^/(g a1) - (a3/a1) w- - (a2/a1) w
      cfh[nf + j] = 1.0 / (g[j] * a1);
      cfh[2 * nf + j] = -a2 / a1;
      step[j] = c[j] * eta[j];
    }
    bool anyu = false;
    for (int v : upd) anyu |= v != 0;
    if (anyu) {
      if (upd != p->mask_h && (rc = set_mask(upd))) return rc;
      if ((rc = comb(iw0, BVk(iz), BPk(iz), BVk(iw), BPk(iw)))) return rc;
      for (int j = 0; j < nf; ++j) {
        cfh[j] = 1.0;                                       // x += c eta w+
        cfh[nf + j] = step[j];
        cfh[2 * nf + j] = 0.0;
      }
      if ((rc = comb(-1, BVk(iw0), BPk(iw0), nullptr, nullptr))) return rc;
    }
    ++total;
    for (int j = 0; j < nf; ++j) {
      if (!upd[j]) continue;
      eta[j] = -sn[j] * eta[j];
      its[j]++;
      if (std::fabs(eta[j]) <= p->o.inner_tol * g1[j] || !(g2[j] > 0)) done[j] = 1;
      g0[j] = g[j];
      g[j] = gn[j];
    }
    // rotate: v- <- v <- v+, z^ <- z^+, w- <-> w (w+ was written over w-)
    const int t = iv0;
    iv0 = iv;
    iv = iv1;
    iv1 = t;
    std::swap(iz, iz1);
    std::swap(iw0, iw);
  }
  p->cur_mask = nullptr;
  for (MGPlan* m : {&p->mgW, &p->mgK, &p->mgQ, &p->mgQH}) { m->mask = nullptr; m->active = m->nb; }
  p->last_its = its;
  if ((int)p->its_acc.size() != nf) p->its_acc.assign(nf, 0);
  {
    // model: per frequency, each step applies the block preconditioner and
    // the block product and makes 15 vector passes (two dots, three updates)
    const double per_j_block = p->model_block / nf, per_j_bmat = p->model_bmat / nf, fv = p->model_fvec / nf;
    for (int j = 0; j < nf; ++j) {
      if (!p->freq_on[j]) continue;
      const double kk = its[j];
      p->bytes_acc += (kk + 1.0) * per_j_block + kk * per_j_bmat + (15.0 * kk + 4.0) * fv;
    }
  }
  for (int j = 0; j < nf; ++j) {
    if (!p->freq_on[j]) continue;
    p->its_acc[j] += its[j];
    p->inner_its_sum += its[j];
    p->inner_blocks += 1;
    p->inner_its_max = std::max(p->inner_its_max, its[j]);
  }
  return PINTOC_OK;
}

// The block-circulant preconditioner: FFT in time (+ T_l^{-1} for Stokes),
// per-frequency block solves (one application of P~_j / P~_j^(UZ), or GMRES
// to the inner tolerance), (T_r^{-1} +) inverse FFT.  Stokes: Algorithms 1
// and 2; Oseen: Algorithm 3 and its GMRES wrapper (section 4).
template <typename R>
static int precond_apply_t(pintoc_problem* p, const double* const* r, double* const* z, hipStream_t s) {
  cpx<R>*Vb = (cpx<R>*)p->Vb, *Vx = (cpx<R>*)p->Vx, *Pb = (cpx<R>*)p->Pb, *Px = (cpx<R>*)p->Px;
  const int mode = p->d.flow == PINTOC_STOKES ? 1 : 0;
  int ph = phase_open(p, s, PINTOC_PHASE_FFT);
  for (size_t k = 0; k < p->mem.size(); ++k) {
    if (!p->mem_on[k]) continue;
    const Member& mb = p->mem[k];
    launch_time_fft_fwd<R>(s, r[k], Vb + (size_t)mb.f0 * p->segV, Pb + (size_t)mb.f0 * p->segP, mb.nt, p->L, p->nq2,
                           p->np2, p->tw + mb.tw0, p->tj + mb.f0, mb.tau, mode);
  }
  phase_close(p, s, ph);
  ph = phase_open(p, s, PINTOC_PHASE_BLOCKS);
  if (p->o.inner == PINTOC_INNER_LINEAR) {
    int rc = member_mask(p, s);                // group members that sit out skip every block kernel
    if (rc) return rc;
    block_precond<R>(p, s, Vb, Pb, Vx, Px);
    clear_member_mask(p);
    p->bytes_acc += p->model_block * active_fraction(p);
  } else {
    int rc = p->o.inner == PINTOC_INNER_MINRES ? minres_blocks<R>(p, s) : gmres_blocks<R>(p, s);
    if (rc) return rc;
  }
  phase_close(p, s, ph);
  ph = phase_open(p, s, PINTOC_PHASE_IFFT);
  for (size_t k = 0; k < p->mem.size(); ++k) {
    if (!p->mem_on[k]) continue;
    const Member& mb = p->mem[k];
    launch_time_fft_inv<R>(s, Vx + (size_t)mb.f0 * p->segV, Px + (size_t)mb.f0 * p->segP, z[k], mb.nt, p->L, p->nq2,
                           p->np2, p->tw + mb.tw0, p->tj + mb.f0, mb.tau, mode);
  }
  phase_close(p, s, ph);
  p->bytes_acc += p->model_fft * active_fraction(p);
  return PINTOC_OK;
}

// z_k = P^{-1} r_k for the members k with r[k] != NULL, in one fused
// application (a lone problem: its one vector)
static int precond_members(pintoc_problem* p, const double* const* r, double* const* z, hipStream_t s) {
  const size_t nm = p->mem.size();
  std::vector<const double*> rr(r, r + nm);
  for (size_t k = 0; k < nm; ++k) p->mem_on[k] = r[k] != nullptr;
  for (size_t k = 0; k < nm; ++k)
    for (int j = 0; j < p->mem[k].nf; ++j) p->freq_on[p->mem[k].f0 + j] = p->mem_on[k];
  // on a square of side l: P^{-1} = D_c^{-1} P'^{-1} D_r^{-1} (see create_impl; lone problems only)
  const double l = p->side;
  if (l != 1.0) {
    launch_scale_canon(s, p->dscale, rr[0], p->d.N, p->d.nt, 1.0 / (l * l), 1.0 / l);
    rr[0] = p->dscale;
  }
  int rc = p->o.precision == PINTOC_PREC_FP64 ? precond_apply_t<double>(p, rr.data(), z, s)
                                              : precond_apply_t<float>(p, rr.data(), z, s);
  std::fill(p->mem_on.begin(), p->mem_on.end(), 1);
  std::fill(p->freq_on.begin(), p->freq_on.end(), 1);
  if (rc) return rc;
  if (l != 1.0) launch_scale_canon(s, z[0], z[0], p->d.N, p->d.nt, 1.0, l);
  p->precond_apps++;
  HIPCHK(hipGetLastError());
  return PINTOC_OK;
}

static int precond(pintoc_problem* p, const double* r, double* z, hipStream_t s) {
  return precond_members(p, &r, &z, s);
}

// ------------------------------------------------------------ public entries
static int check_bound(pintoc_problem* p) {
  if (!p) return fail(PINTOC_EINVAL, "NULL handle");
  if (!p->bound) return fail(PINTOC_ESTATE, "no workspace bound (or its scratch binding was taken over)");
  return PINTOC_OK;
}

static int check_ready(pintoc_problem* p) {
  const int rc = check_bound(p);
  if (rc) return rc;
  if (p->group) return fail(PINTOC_EINVAL, "a group handle takes the pintoc_group_* entry points");
  return PINTOC_OK;
}

extern "C" int pintoc_assemble_rhs(pintoc_problem* p, const double* vd, double* b, void* stream) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!vd || !b) return fail(PINTOC_EINVAL, "NULL vector");
  launch_assemble_rhs((hipStream_t)stream, vd, b, p->d.N, p->d.nt, p->tau);
  if (p->side != 1.0) launch_scale_canon((hipStream_t)stream, b, b, p->d.N, p->d.nt, p->side * p->side, p->side);
  HIPCHK(hipGetLastError());
  return PINTOC_OK;
}

extern "C" int pintoc_assemble_rhs_data(pintoc_problem* p, const double* vd, const double* f, const double* h,
                                        const double* v0, double* b, void* stream) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!b) return fail(PINTOC_EINVAL, "NULL right-hand side");
  hipStream_t s = (hipStream_t)stream;
  // the unit-square equivalent's right-hand side, then D_r (see pintoc_problem_create)
  launch_rhs_data(s, vd, f, h, v0, b, p->d.N, p->d.nt, p->tau, p->d.nu,
                  p->d.flow == PINTOC_OSEEN ? p->conv50 : nullptr);
  if (p->side != 1.0) launch_scale_canon(s, b, b, p->d.N, p->d.nt, p->side * p->side, p->side);
  HIPCHK(hipGetLastError());
  return PINTOC_OK;
}

// y = A x of member k
static void kkt_member(pintoc_problem* p, int k, const double* x, double* y, hipStream_t s) {
  const Member& mb = p->mem[k];
  // on a square of side l: A = D_r A' D_c (see create_impl)
  const double l = p->side;
  if (l != 1.0) {
    launch_scale_canon(s, p->dscale, x, p->d.N, mb.nt, 1.0, 1.0 / l);
    x = p->dscale;
  }
  launch_kkt_apply(s, x, y, p->d.N, mb.nt, mb.tau, mb.beta, mb.nu, p->d.flow == PINTOC_OSEEN ? p->conv50t : nullptr);
  if (l != 1.0) launch_scale_canon(s, y, y, p->d.N, mb.nt, l * l, l);
}

static void kkt(pintoc_problem* p, const double* x, double* y, hipStream_t s) { kkt_member(p, 0, x, y, s); }

// the all-at-once product inside a solve: timed as its phase, counted in the byte model
static void kkt_t(pintoc_problem* p, const double* x, double* y, hipStream_t s, int k = 0) {
  const int ph = phase_open(p, s, PINTOC_PHASE_MATVEC);
  kkt_member(p, k, x, y, s);
  phase_close(p, s, ph);
  p->bytes_acc += 2.0 * 8.0 * (double)p->mem[k].n_all;
}

extern "C" int pintoc_kkt_apply(pintoc_problem* p, const double* x, double* y, void* stream) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!x || !y || x == y) return fail(PINTOC_EINVAL, "NULL or aliased vectors");
  kkt(p, x, y, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return PINTOC_OK;
}

extern "C" int pintoc_precond_apply(pintoc_problem* p, const double* r, double* z, void* stream) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!r || !z || r == z) return fail(PINTOC_EINVAL, "NULL or aliased vectors");
  return precond(p, r, z, (hipStream_t)stream);
}

// dots of the first k vectors of V (stride n) with w, returned on the host
static int dots(pintoc_problem* p, hipStream_t s, const double* V, int k, const double* w, double* dev_out,
                double* host_out, size_t n = 0) {
  if (n == 0) n = (size_t)p->n_all;
  launch_mdot(s, V, n, k, w, n, p->part, dev_out);
  HIPCHK(hipMemcpyAsync(host_out, dev_out, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return PINTOC_OK;
}

// Preconditioned MINRES (Paige & Saunders) on the symmetric all-at-once
// matrix with the symmetric positive definite linear preconditioner of
// Algorithm 1 (section 3.3), FP64, from the iterate in x.  Lanczos in the
// preconditioner's inner product: z_j = P^{-1} v_j / gamma_j with
// gamma_j^2 = <P^{-1} v_j, v_j>, delta_j = <A z_j, z_j>,
// v_{j+1} = A z_j - (delta_j / gamma_j) v_j - (gamma_j / gamma_{j-1}) v_{j-1};
// the tridiagonal matrix is reduced by Givens rotations (c, s) and x moves
// along w_{j+1} = (z_j - a3 w_{j-1} - a2 w_j) / a1.  |eta| is the residual norm
// in the preconditioner's inner product.  The true residual decides the stop:
// it is formed every kMinresCheck steps once |eta| <= 100 tol |eta_0| and at
// every step with |eta| <= tol |eta_0|.  A breakdown of the recurrence starts
// it again from x.  Vectors: v_{j-1}, v_j, w_{j-1}, w_j, A z in the FGMRES
// basis V, z_j and P^{-1} v_{j+1} in Z.  Returns PINTOC_OK or an error; its,
// res (true residual norm) and conv report the outcome.
constexpr int kMinresCheck = 5;

static int solve_minres(pintoc_problem* p, const double* b, double* x, double bnorm, hipStream_t s, int& its,
                        double& res, bool& conv, std::vector<double>& hist) {
  const size_t n = (size_t)p->n_all;
  double hb[2];
  int rc;
  double* V[2] = {p->Vk, p->Vk + n};                       // v_{j-1} (then v_{j+1}), v_j
  double* Wv[2] = {p->Vk + 2 * n, p->Vk + 3 * n};          // w_{j-1} (then w_{j+1}), w_j
  double* AZ = p->Vk + 4 * n;
  auto true_residual = [&]() -> int {
    kkt_t(p, x, p->rvec, s);
    launch_axpby(s, p->rvec, b, 1.0, -1.0, n);
    int r = dots(p, s, p->rvec, 1, p->rvec, p->dd, hb);
    res = std::sqrt(hb[0]);
    return r;
  };
  if ((rc = true_residual())) return rc;
  while (true) {
    if (!std::isfinite(res)) return PINTOC_OK;
    if (res <= p->o.tol * bnorm) { conv = true; return PINTOC_OK; }
    if (its >= p->o.max_outer) return PINTOC_OK;
    double* Zc = p->Zk;                                    // z_j
    double* Zn = p->Zk + n;                                // P^{-1} v_{j+1}
    // v_1 = r, z = P^{-1} v_1, gamma_1 = sqrt(<z, v_1>)
    launch_axpby(s, V[1], p->rvec, 1.0, 0.0, n);
    if ((rc = precond(p, V[1], Zc, s))) return rc;
    if ((rc = dots(p, s, V[1], 1, Zc, p->dd, hb))) return rc;
    if (!(hb[0] > 0)) return PINTOC_OK;                    // not positive definite
    double g = std::sqrt(hb[0]), g_old = 1.0;
    const double g1 = g;
    double eta = g, c_old = 1.0, c = 1.0, s_old = 0.0, sn = 0.0;
    launch_fill_zero(s, V[0], n * sizeof(double));
    launch_fill_zero(s, Wv[0], n * sizeof(double));
    launch_fill_zero(s, Wv[1], n * sizeof(double));
    const int its0 = its;
    bool checked = false;
    while (its < p->o.max_outer) {
      launch_axpby(s, Zc, Zc, 1.0 / g, 0.0, n);             // z_j
      kkt_t(p, Zc, AZ, s);
      p->bytes_acc += 14.0 * p->model_canon;                // vector updates and dots of one step
      if ((rc = dots(p, s, AZ, 1, Zc, p->dd, hb))) return rc;
      const double delta = hb[0];
      // v_{j+1} over v_{j-1}
      launch_axpbypcz(s, V[0], AZ, V[1], 1.0, -delta / g, -g / g_old, n);
      if ((rc = precond(p, V[0], Zn, s))) return rc;
      if ((rc = dots(p, s, V[0], 1, Zn, p->dd, hb))) return rc;
      const double g2 = hb[0];
      const double g_new = std::sqrt(std::max(g2, 0.0));
      const double a0 = c * delta - c_old * sn * g;
      const double a1 = std::hypot(a0, g_new);
      const double a2 = sn * delta + c_old * c * g;
      const double a3 = s_old * g;
      if (!(a1 > 0) || !std::isfinite(a1)) break;
      c_old = c;
      s_old = sn;
      c = a0 / a1;
      sn = g_new / a1;
      // w_{j+1} over w_{j-1}, then x += c eta w_{j+1}
      launch_axpbypcz(s, Wv[0], Zc, Wv[1], 1.0 / a1, -a2 / a1, -a3 / a1, n);
      launch_axpby(s, x, Wv[0], c * eta, 1.0, n);
      eta = -sn * eta;
      ++its;
      const double e = std::fabs(eta);
      hist.push_back(e / g1);
      checked = false;
      if (e <= p->o.tol * g1 || (e <= 100.0 * p->o.tol * g1 && (its - its0) % kMinresCheck == 0)) {
        if ((rc = true_residual())) return rc;
        checked = true;
        if (res <= p->o.tol * bnorm) { conv = true; return PINTOC_OK; }
      }
      if (!(g2 > 0)) break;
      std::swap(V[0], V[1]);
      std::swap(Wv[0], Wv[1]);
      std::swap(Zc, Zn);
      g_old = g;
      g = g_new;
    }
    // breakdown or the iteration cap: start again from x (the loop head stops at the cap)
    const double prev = res;
    if (!checked && (rc = true_residual())) return rc;
    if (its == its0 || !(res < prev || checked)) return PINTOC_OK;
  }
}

// FGMRES in the frequency domain (section 3.1, Theorem 1): the Krylov vectors
// are the scaled kept-frequency spectra (freq_kernels.hip); the operator is
// A^ = diag(G_j) + corner term, the preconditioner the block solves alone, so
// neither needs an FFT: b is transformed once at the start and x once at the
// end.  The operations and stopping rule are those of pintoc_solve's FGMRES;
// the reported residual is the time-domain one of the transformed-back x.
static void matvec_freq(pintoc_problem* p, const double* x, double* y, hipStream_t s) {
  const int ph = phase_open(p, s, PINTOC_PHASE_MATVEC);
  const int nf = p->nf;
  const double2 *xV = (const double2*)x, *xP = xV + (size_t)nf * p->segV;
  double2 *yV = (double2*)y, *yP = yV + (size_t)nf * p->segV;
  const bool oseen = p->d.flow == PINTOC_OSEEN;
  launch_block_mat<double>(s, yV, yP, xV, xP, p->d.N, nf, oseen ? p->bc : p->gcoef,
                           oseen ? (const double*)p->tconv[0][0] : nullptr,
                           oseen ? (const double*)p->tconv[1][0] : nullptr, kAll);
  launch_freq_corner(s, yV, xV, p->ftmp, p->fsc, p->d.N, nf, p->d.nt);
  phase_close(p, s, ph);
  p->bytes_acc += 2.0 * 8.0 * (double)p->nF + 3.0 * 0.5 * 8.0 * (double)p->nF;
}

template <typename R>
static int precond_freq_t(pintoc_problem* p, const double* v, double* z, hipStream_t s) {
  cpx<R>*Vb = (cpx<R>*)p->Vb, *Vx = (cpx<R>*)p->Vx, *Pb = (cpx<R>*)p->Pb, *Px = (cpx<R>*)p->Px;
  const int mode = p->d.flow == PINTOC_STOKES ? 1 : 0;
  int ph = phase_open(p, s, PINTOC_PHASE_FFT);           // the T_l^{-1} transform in place of the FFT
  launch_freq_convert<R>(s, (const double2*)v, Vb, Pb, nullptr, p->nf, p->nq2, p->np2, p->tj, p->tau, mode, 0);
  phase_close(p, s, ph);
  ph = phase_open(p, s, PINTOC_PHASE_BLOCKS);
  if (p->o.inner == PINTOC_INNER_LINEAR) {
    block_precond<R>(p, s, Vb, Pb, Vx, Px);
    p->bytes_acc += p->model_block;
  } else {
    int rc = p->o.inner == PINTOC_INNER_MINRES ? minres_blocks<R>(p, s) : gmres_blocks<R>(p, s);
    if (rc) return rc;
  }
  phase_close(p, s, ph);
  ph = phase_open(p, s, PINTOC_PHASE_IFFT);
  launch_freq_convert<R>(s, nullptr, Vx, Px, (double2*)z, p->nf, p->nq2, p->np2, p->tj, p->tau, mode, 1);
  phase_close(p, s, ph);
  p->bytes_acc += 2.0 * (p->model_fvec + 8.0 * (double)p->nF);
  p->precond_apps++;
  HIPCHK(hipGetLastError());
  return PINTOC_OK;
}

static int precond_freq(pintoc_problem* p, const double* v, double* z, hipStream_t s) {
  return p->o.precision == PINTOC_PREC_FP64 ? precond_freq_t<double>(p, v, z, s) : precond_freq_t<float>(p, v, z, s);
}

static int solve_freq(pintoc_problem* p, const double* b, double* x, double bnorm, hipStream_t s, int& its,
                      double& res, bool& conv, std::vector<double>& hist) {
  const size_t n = (size_t)p->nF;
  const int m = p->o.restart, nf = p->nf;
  const Member& mb = p->mem[0];
  double hb[64], hb2[64];
  int rc;
  // b~ = s F b and x~ = s F x (forward FFT without the T transforms)
  double2 *fb = (double2*)p->fb, *fx = (double2*)mb.xtmp;
  int ph = phase_open(p, s, PINTOC_PHASE_FFT);
  launch_time_fft_fwd<double>(s, b, fb, fb + (size_t)nf * p->segV, mb.nt, p->L, p->nq2, p->np2, p->tw, p->tj, mb.tau, 0);
  launch_freq_scale(s, fb, fb, p->fsc, nf, p->segV, p->segP);
  launch_time_fft_fwd<double>(s, x, fx, fx + (size_t)nf * p->segV, mb.nt, p->L, p->nq2, p->np2, p->tw, p->tj, mb.tau, 0);
  launch_freq_scale(s, fx, fx, p->fsc, nf, p->segV, p->segP);
  phase_close(p, s, ph);
  double* rv = mb.rvec;
  double* xf = mb.xtmp;
  auto residual = [&]() -> int {                         // r~ = b~ - A^ x~, res = ||r~||
    matvec_freq(p, xf, rv, s);
    launch_axpby(s, rv, p->fb, 1.0, -1.0, n);
    int r = dots(p, s, rv, 1, rv, p->dd, hb, n);
    if (r) return r;
    res = std::sqrt(hb[0]);
    return PINTOC_OK;
  };
  if ((rc = residual())) return rc;
  const double res0 = res;
  bool stalled = false;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  while (true) {
    if (!std::isfinite(res)) break;
    if (res <= p->o.tol * bnorm) { conv = true; break; }
    if (its >= p->o.max_outer) break;
    launch_axpby(s, mb.Vk, rv, 1.0 / res, 0.0, n);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = res;
    int k = 0;
    bool breakdown = false;
    for (; k < m && its < p->o.max_outer; ++k) {
      double* vk = mb.Vk + (size_t)k * n;
      double* zk = mb.Zk + (size_t)k * n;
      double* w = mb.Vk + (size_t)(k + 1) * n;
      if ((rc = precond_freq(p, vk, zk, s))) return rc;
      matvec_freq(p, zk, w, s);
      const int ph2 = phase_open(p, s, PINTOC_PHASE_ORTH);
      p->bytes_acc += (4.0 * k + 13.0) * 8.0 * (double)n;
      if ((rc = dots(p, s, mb.Vk, k + 1, w, p->dd, hb, n))) return rc;
      launch_mgs_update(s, w, mb.Vk, n, k + 1, p->dd, n);
      if ((rc = dots(p, s, mb.Vk, k + 1, w, p->dd2, hb2, n))) return rc;
      launch_mgs_update(s, w, mb.Vk, n, k + 1, p->dd2, n);
      double nrm2;
      if ((rc = dots(p, s, w, 1, w, p->dd, &nrm2, n))) return rc;
      const double hk1 = std::sqrt(nrm2);
      for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = hb[i] + hb2[i];
      H[(size_t)(k + 1) * m + k] = hk1;
      if (hk1 > 0) launch_axpby(s, w, w, 1.0 / hk1, 0.0, n);
      else breakdown = true;
      phase_close(p, s, ph2);
      for (int i = 0; i < k; ++i) {
        const double a = H[(size_t)i * m + k], c = H[(size_t)(i + 1) * m + k];
        H[(size_t)i * m + k] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)k * m + k], c = H[(size_t)(k + 1) * m + k];
      const double t = std::hypot(a, c);
      cs[k] = t > 0 ? a / t : 1.0;
      sn[k] = t > 0 ? c / t : 0.0;
      H[(size_t)k * m + k] = t;
      H[(size_t)(k + 1) * m + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      ++its;
      hist.push_back(std::fabs(g[k + 1]) / bnorm);
      stalled = p->o.stall_guard && its >= std::max(10, m) && std::fabs(g[k + 1]) > 0.5 * res0;
      if (std::fabs(g[k + 1]) <= p->o.tol * bnorm || breakdown || stalled) { ++k; break; }
    }
    for (int i = k - 1; i >= 0; --i) {
      double v = g[i];
      for (int j = i + 1; j < k; ++j) v -= H[(size_t)i * m + j] * y[j];
      y[i] = v / H[(size_t)i * m + i];
    }
    const int ph3 = phase_open(p, s, PINTOC_PHASE_ORTH);
    HIPCHK(hipMemcpyAsync(p->dd, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    launch_lincomb_add(s, xf, mb.Zk, n, k, p->dd, n);
    phase_close(p, s, ph3);
    p->bytes_acc += (k + 2.0 + 4.0) * 8.0 * (double)n;
    if ((rc = residual())) return rc;
    if ((breakdown || stalled) && !(res <= p->o.tol * bnorm)) break;
  }
  // x = F^{-1} (x~ / s), then the time-domain true residual
  ph = phase_open(p, s, PINTOC_PHASE_IFFT);
  launch_freq_scale(s, (double2*)rv, (const double2*)xf, p->fisc, nf, p->segV, p->segP);
  launch_time_fft_inv<double>(s, (const double2*)rv, (const double2*)rv + (size_t)nf * p->segV, x, mb.nt, p->L,
                              p->nq2, p->np2, p->tw, p->tj, mb.tau, 0);
  phase_close(p, s, ph);
  double* rt = mb.Zk;                                      // a time-domain vector's worth of scratch
  kkt_t(p, x, rt, s);
  launch_axpby(s, rt, b, 1.0, -1.0, (size_t)p->n_all);
  if ((rc = dots(p, s, rt, 1, rt, p->dd, hb))) return rc;
  res = std::sqrt(hb[0]);
  conv = res <= p->o.tol * bnorm;
  return PINTOC_OK;
}

extern "C" int pintoc_solve(pintoc_problem* p, const double* b, double* x, pintoc_solve_stats* st, void* stream) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!b || !x || b == x) return fail(PINTOC_EINVAL, "NULL or aliased vectors");
  hipStream_t s = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  const size_t n = (size_t)p->n_all;
  const int m = p->o.restart;
  const int budget = st ? st->cycle_budget : 0;
  const bool resume = st && st->resume;
  auto& pz = p->paused;
  std::chrono::steady_clock::duration prev_elapsed{};
  double prev_phase[PINTOC_NPHASES] = {};
  if (resume) {
    if (!pz.on) return fail(PINTOC_ESTATE, "no paused solve to resume");
    prev_elapsed = pz.elapsed;
    std::copy(pz.phase, pz.phase + PINTOC_NPHASES, prev_phase);
    if (pz.b != b || pz.x != x) return fail(PINTOC_EINVAL, "a resumed solve must pass the paused call's b and x");
    if (p->o.outer != PINTOC_OUTER_FGMRES) return fail(PINTOC_EINVAL, "only FGMRES solves can be paused");
  } else {
    if (budget < 0 || (budget > 0 && p->o.outer != PINTOC_OUTER_FGMRES))
      return fail(PINTOC_EINVAL, "cycle_budget needs FGMRES and must be >= 0");
    pz = pintoc_problem::Paused{};
    p->precond_apps = 0;
    p->inner_its_sum = 0;
    p->inner_blocks = 0;
    p->inner_its_max = 0;
    p->bytes_acc = 0.0;
    p->its_acc.assign(p->nf, 0);
  }
  p->pt.used = 0;
  p->pt.on = true;
  struct TimerOff {
    pintoc_problem* q;
    ~TimerOff() { q->pt.on = false; }
  } timer_off{p};
  std::vector<double> hist = resume ? pz.hist : std::vector<double>();
  double hb[64], hb2[64];
  double bnorm;
  if (resume) {
    bnorm = pz.bnorm;
  } else {
    if ((rc = dots(p, s, b, 1, b, p->dd, hb))) return rc;
    bnorm = std::sqrt(hb[0]);
  }
  int its = resume ? pz.its : 0;
  double res = 0;
  bool conv = false, paused = false;
  pz.on = false;
  if (bnorm == 0.0) {
    launch_fill_zero(s, x, n * sizeof(double));
    conv = true;
  } else if (p->o.outer == PINTOC_OUTER_MINRES) {
    if ((rc = solve_minres(p, b, x, bnorm, s, its, res, conv, hist))) return rc;
  } else if (p->o.outer == PINTOC_OUTER_FGMRES_FREQ) {
    if ((rc = solve_freq(p, b, x, bnorm, s, its, res, conv, hist))) return rc;
  } else {
    // r = b - A x
    kkt_t(p, x, p->rvec, s);
    launch_axpby(s, p->rvec, b, 1.0, -1.0, n);
    if ((rc = dots(p, s, p->rvec, 1, p->rvec, p->dd, hb))) return rc;
    res = std::sqrt(hb[0]);
    const double res0 = resume ? pz.res0 : res;
    bool stalled = false;
    int cycles = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    while (true) {
      if (!std::isfinite(res)) break;                  // NaN or overflow: give up
      if (res <= p->o.tol * bnorm) { conv = true; break; }
      if (its >= p->o.max_outer) break;
      if (budget > 0 && cycles >= budget) {            // pause at a restart boundary
        paused = true;
        pz.on = true;
        pz.b = b;
        pz.x = x;
        pz.its = its;
        pz.bnorm = bnorm;
        pz.res0 = res0;
        pz.hist = hist;
        break;
      }
      ++cycles;
      // V_0 = r / ||r||
      launch_axpby(s, p->Vk, p->rvec, 1.0 / res, 0.0, n);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = res;
      int k = 0;
      bool breakdown = false;
      for (; k < m && its < p->o.max_outer; ++k) {
        const Member& m0 = p->mem[0];
        double* vk = p->Vk + (size_t)k * n;
        double* zk = m0.Zk32 ? m0.xtmp : p->Zk + (size_t)k * n;
        double* w = p->Vk + (size_t)(k + 1) * n;
        if ((rc = precond(p, vk, zk, s))) return rc;
        kkt_t(p, zk, w, s);
        if (m0.Zk32) {
          launch_to_f32(s, m0.Zk32 + (size_t)k * n, zk, n);
          p->bytes_acc += 1.5 * p->model_canon;
        }
        // classical Gram-Schmidt, twice
        const int ph = phase_open(p, s, PINTOC_PHASE_ORTH);
        p->bytes_acc += (4.0 * k + 13.0) * p->model_canon;
        if ((rc = dots(p, s, p->Vk, k + 1, w, p->dd, hb))) return rc;
        launch_mgs_update(s, w, p->Vk, n, k + 1, p->dd, n);
        if ((rc = dots(p, s, p->Vk, k + 1, w, p->dd2, hb2))) return rc;
        launch_mgs_update(s, w, p->Vk, n, k + 1, p->dd2, n);
        double nrm2;
        if ((rc = dots(p, s, w, 1, w, p->dd, &nrm2))) return rc;
        const double hk1 = std::sqrt(nrm2);
        for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = hb[i] + hb2[i];
        H[(size_t)(k + 1) * m + k] = hk1;
        if (hk1 > 0) launch_axpby(s, w, w, 1.0 / hk1, 0.0, n);
        else breakdown = true;
        phase_close(p, s, ph);
        for (int i = 0; i < k; ++i) {
          const double a = H[(size_t)i * m + k], c = H[(size_t)(i + 1) * m + k];
          H[(size_t)i * m + k] = cs[i] * a + sn[i] * c;
          H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * c;
        }
        const double a = H[(size_t)k * m + k], c = H[(size_t)(k + 1) * m + k];
        const double t = std::hypot(a, c);
        cs[k] = t > 0 ? a / t : 1.0;
        sn[k] = t > 0 ? c / t : 0.0;
        H[(size_t)k * m + k] = t;
        H[(size_t)(k + 1) * m + k] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        ++its;
        hist.push_back(std::fabs(g[k + 1]) / bnorm);
        // stagnation guard: a first restart cycle (at least ten iterations)
        // without halving the initial residual
        stalled = p->o.stall_guard && its >= std::max(10, m) && std::fabs(g[k + 1]) > 0.5 * res0;
        if (std::fabs(g[k + 1]) <= p->o.tol * bnorm || breakdown || stalled) { ++k; break; }
      }
      // y = H^{-1} g (upper triangular), x += Z y
      for (int i = k - 1; i >= 0; --i) {
        double v = g[i];
        for (int j = i + 1; j < k; ++j) v -= H[(size_t)i * m + j] * y[j];
        y[i] = v / H[(size_t)i * m + i];
      }
      const int ph = phase_open(p, s, PINTOC_PHASE_ORTH);
      HIPCHK(hipMemcpyAsync(p->dd, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
      if (p->mem[0].Zk32)
        launch_lincomb_add_f32(s, x, p->mem[0].Zk32, n, k, p->dd, n);
      else
        launch_lincomb_add(s, x, p->Zk, n, k, p->dd, n);
      phase_close(p, s, ph);
      p->bytes_acc += ((p->mem[0].Zk32 ? 0.5 : 1.0) * k + 2.0 + 4.0) * p->model_canon;
      // true residual
      kkt_t(p, x, p->rvec, s);
      launch_axpby(s, p->rvec, b, 1.0, -1.0, n);
      if ((rc = dots(p, s, p->rvec, 1, p->rvec, p->dd, hb))) return rc;
      res = std::sqrt(hb[0]);
      if ((breakdown || stalled) && !(res <= p->o.tol * bnorm)) break;
    }
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (st) {
    double* hist_out = st->residual_history;
    const int hcap = st->history_capacity;
    int32_t* cnt_out = st->inner_counts;
    const int ccap = st->inner_counts_capacity;
    std::memset(st, 0, sizeof(*st));
    st->residual_history = hist_out;
    st->history_capacity = hcap;
    st->inner_counts = cnt_out;
    st->inner_counts_capacity = ccap;
    if (hist_out && hcap > 0) {
      st->history_length = (int32_t)std::min<size_t>((size_t)hcap, hist.size());
      std::copy(hist.begin(), hist.begin() + st->history_length, hist_out);
    }
    if (cnt_out && ccap > 0)
      for (int j = 0; j < std::min(ccap, p->nf); ++j) cnt_out[j] = (int32_t)p->its_acc[j];
    phase_sum(p, st->phase_seconds);
    const auto el = std::chrono::steady_clock::now() - t0 + prev_elapsed;
    for (int i = 0; i < PINTOC_NPHASES; ++i) st->phase_seconds[i] += prev_phase[i];
    if (paused) {
      pz.elapsed = el;
      for (int i = 0; i < PINTOC_NPHASES; ++i) pz.phase[i] = st->phase_seconds[i];
    }
    st->model_bytes = p->bytes_acc;
    st->precond_model_bytes = p->model_fft + p->model_block;
    st->outer_iterations = its;
    st->converged = conv ? 1 : 0;
    st->rel_residual = bnorm > 0 ? res / bnorm : 0.0;
    st->precond_applications = p->precond_apps;
    st->inner_iterations_mean = p->inner_blocks ? (double)p->inner_its_sum / p->inner_blocks : 0.0;
    st->inner_iterations_max = p->inner_its_max;
    st->seconds = std::chrono::duration<double>(el).count();
    st->cycle_budget = budget;
    st->resume = resume ? 1 : 0;
  }
  if (paused) return PINTOC_PAUSED;
  return conv ? PINTOC_OK : PINTOC_NOT_CONVERGED;
}

// Several problems at once: one host thread per problem, each driving its
// problem's solve on that problem's stream.
// ------------------------------------------------------------ groups
// A group solves the all-at-once systems of several problems that share N,
// the flow, the wind and the options.  Every member runs its own restarted
// FGMRES with the operations of pintoc_solve in the same order; the members
// advance in lockstep, and the preconditioner applications of all members
// still iterating are one fused application (their kept frequencies form one
// batch of every per-frequency kernel).  Each kernel and reduction acts on
// one member's data in a fixed order, so every member's iterates equal those
// of a lone solve bit for bit.
struct MemberSolve {
  double bnorm = 0, res = 0, res0 = 0;
  int its = 0, k = 0, apps = 0, inner_max = 0;
  bool done = false, conv = false, in_cycle = false, stalled = false, breakdown = false;
  std::vector<double> H, cs, sn, g, y, hist;
};

static int check_member(pintoc_problem* p, int32_t k) {
  const int rc = check_bound(p);
  if (rc) return rc;
  if (k < 0 || k >= (int32_t)p->mem.size()) return fail(PINTOC_EINVAL, "member index out of range");
  return PINTOC_OK;
}

extern "C" int32_t pintoc_group_size(const pintoc_problem* p) { return p ? (int32_t)p->mem.size() : 0; }

extern "C" int64_t pintoc_group_vector_length(const pintoc_problem* p, int32_t k) {
  return (p && k >= 0 && k < (int32_t)p->mem.size()) ? p->mem[k].n_all : 0;
}

extern "C" int pintoc_group_assemble_rhs(pintoc_problem* p, int32_t k, const double* vd, double* b, void* stream) {
  int rc = check_member(p, k);
  if (rc) return rc;
  if (!vd || !b) return fail(PINTOC_EINVAL, "NULL vector");
  launch_assemble_rhs((hipStream_t)stream, vd, b, p->d.N, p->mem[k].nt, p->mem[k].tau);
  HIPCHK(hipGetLastError());
  return PINTOC_OK;
}

extern "C" int pintoc_group_kkt_apply(pintoc_problem* p, int32_t k, const double* x, double* y, void* stream) {
  int rc = check_member(p, k);
  if (rc) return rc;
  if (!x || !y || x == y) return fail(PINTOC_EINVAL, "NULL or aliased vectors");
  kkt_member(p, k, x, y, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return PINTOC_OK;
}

extern "C" int pintoc_group_precond_apply(pintoc_problem* p, const double* const* r, double* const* z, void* stream) {
  int rc = check_bound(p);
  if (rc) return rc;
  if (!r || !z) return fail(PINTOC_EINVAL, "NULL vector arrays");
  for (size_t k = 0; k < p->mem.size(); ++k)
    if (r[k] && (!z[k] || r[k] == z[k])) return fail(PINTOC_EINVAL, "member " + std::to_string(k) + ": NULL or aliased output");
  return precond_members(p, r, z, (hipStream_t)stream);
}

extern "C" int pintoc_group_solve(pintoc_problem* p, const double* const* b, double* const* x, pintoc_solve_stats* st,
                                  void* stream) {
  int rc = check_bound(p);
  if (rc) return rc;
  if (!b || !x) return fail(PINTOC_EINVAL, "NULL vector arrays");
  if (p->o.outer != PINTOC_OUTER_FGMRES) return fail(PINTOC_EINVAL, "a group solves with FGMRES");
  const int nm = (int)p->mem.size();
  for (int k = 0; k < nm; ++k)
    if (!b[k] || !x[k] || b[k] == x[k]) return fail(PINTOC_EINVAL, "member " + std::to_string(k) + ": NULL or aliased vectors");
  hipStream_t s = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  const int m = p->o.restart;
  p->paused = pintoc_problem::Paused{};
  p->precond_apps = 0;
  p->inner_its_sum = 0;
  p->inner_blocks = 0;
  p->inner_its_max = 0;
  p->bytes_acc = 0.0;
  p->its_acc.assign(p->nf, 0);
  p->pt.used = 0;
  p->pt.on = true;
  struct TimerOff {
    pintoc_problem* q;
    ~TimerOff() { q->pt.on = false; }
  } timer_off{p};
  std::vector<MemberSolve> ms(nm);
  double hb[64], hb2[64];
  for (int k = 0; k < nm; ++k) {
    Member& mb = p->mem[k];
    MemberSolve& q = ms[k];
    const size_t n = (size_t)mb.n_all;
    if ((rc = dots(p, s, b[k], 1, b[k], p->dd, hb, n))) return rc;
    q.bnorm = std::sqrt(hb[0]);
    q.H.assign((size_t)(m + 1) * m, 0.0);
    q.cs.assign(m, 0.0); q.sn.assign(m, 0.0); q.g.assign(m + 1, 0.0); q.y.assign(m, 0.0);
    if (q.bnorm == 0.0) {
      launch_fill_zero(s, x[k], n * sizeof(double));
      q.conv = q.done = true;
      continue;
    }
    kkt_t(p, x[k], mb.rvec, s, k);                       // r = b - A x
    launch_axpby(s, mb.rvec, b[k], 1.0, -1.0, n);
    if ((rc = dots(p, s, mb.rvec, 1, mb.rvec, p->dd, hb, n))) return rc;
    q.res = q.res0 = std::sqrt(hb[0]);
  }
  const double tol = p->o.tol;
  std::vector<const double*> rr(nm);
  std::vector<double*> zz(nm);
  while (true) {
    // start a restart cycle for every member between cycles
    for (int k = 0; k < nm; ++k) {
      MemberSolve& q = ms[k];
      if (q.done || q.in_cycle) continue;
      if (!std::isfinite(q.res)) { q.done = true; continue; }
      if (q.res <= tol * q.bnorm) { q.conv = q.done = true; continue; }
      if (q.its >= p->o.max_outer) { q.done = true; continue; }
      const Member& mb = p->mem[k];
      launch_axpby(s, mb.Vk, mb.rvec, 1.0 / q.res, 0.0, (size_t)mb.n_all);
      std::fill(q.g.begin(), q.g.end(), 0.0);
      q.g[0] = q.res;
      q.k = 0;
      q.breakdown = false;
      q.in_cycle = true;
    }
    bool any = false;
    for (int k = 0; k < nm; ++k) {
      const MemberSolve& q = ms[k];
      const Member& mb = p->mem[k];
      const size_t n = (size_t)mb.n_all;
      rr[k] = q.in_cycle ? mb.Vk + (size_t)q.k * n : nullptr;
      zz[k] = q.in_cycle ? (mb.Zk32 ? mb.xtmp : mb.Zk + (size_t)q.k * n) : nullptr;
      any |= q.in_cycle;
    }
    if (!any) break;
    // one fused preconditioner application for every member in a cycle
    if ((rc = precond_members(p, rr.data(), zz.data(), s))) return rc;
    for (int k = 0; k < nm; ++k) {
      MemberSolve& q = ms[k];
      if (!q.in_cycle) continue;
      q.apps++;
      const Member& mb = p->mem[k];
      for (int j = 0; j < mb.nf; ++j)
        if ((size_t)(mb.f0 + j) < p->last_its.size()) q.inner_max = std::max(q.inner_max, p->last_its[mb.f0 + j]);
      const size_t n = (size_t)mb.n_all;
      const int kk = q.k;
      double* zk = mb.Zk32 ? mb.xtmp : mb.Zk + (size_t)kk * n;
      double* w = mb.Vk + (size_t)(kk + 1) * n;
      kkt_t(p, zk, w, s, k);
      if (mb.Zk32) {
        launch_to_f32(s, mb.Zk32 + (size_t)kk * n, zk, n);
        p->bytes_acc += 1.5 * 8.0 * (double)n;
      }
      // classical Gram-Schmidt, twice
      const int ph = phase_open(p, s, PINTOC_PHASE_ORTH);
      p->bytes_acc += (4.0 * kk + 13.0) * 8.0 * (double)n;
      if ((rc = dots(p, s, mb.Vk, kk + 1, w, p->dd, hb, n))) return rc;
      launch_mgs_update(s, w, mb.Vk, n, kk + 1, p->dd, n);
      if ((rc = dots(p, s, mb.Vk, kk + 1, w, p->dd2, hb2, n))) return rc;
      launch_mgs_update(s, w, mb.Vk, n, kk + 1, p->dd2, n);
      double nrm2;
      if ((rc = dots(p, s, w, 1, w, p->dd, &nrm2, n))) return rc;
      const double hk1 = std::sqrt(nrm2);
      std::vector<double>& H = q.H;
      for (int i = 0; i <= kk; ++i) H[(size_t)i * m + kk] = hb[i] + hb2[i];
      H[(size_t)(kk + 1) * m + kk] = hk1;
      if (hk1 > 0) launch_axpby(s, w, w, 1.0 / hk1, 0.0, n);
      else q.breakdown = true;
      phase_close(p, s, ph);
      for (int i = 0; i < kk; ++i) {
        const double a = H[(size_t)i * m + kk], c = H[(size_t)(i + 1) * m + kk];
        H[(size_t)i * m + kk] = q.cs[i] * a + q.sn[i] * c;
        H[(size_t)(i + 1) * m + kk] = -q.sn[i] * a + q.cs[i] * c;
      }
      const double a = H[(size_t)kk * m + kk], c = H[(size_t)(kk + 1) * m + kk];
      const double t = std::hypot(a, c);
      q.cs[kk] = t > 0 ? a / t : 1.0;
      q.sn[kk] = t > 0 ? c / t : 0.0;
      H[(size_t)kk * m + kk] = t;
      H[(size_t)(kk + 1) * m + kk] = 0.0;
      q.g[kk + 1] = -q.sn[kk] * q.g[kk];
      q.g[kk] = q.cs[kk] * q.g[kk];
      ++q.its;
      q.hist.push_back(std::fabs(q.g[kk + 1]) / q.bnorm);
      q.stalled = p->o.stall_guard && q.its >= std::max(10, m) && std::fabs(q.g[kk + 1]) > 0.5 * q.res0;
      const bool stop = std::fabs(q.g[kk + 1]) <= tol * q.bnorm || q.breakdown || q.stalled;
      q.k = kk + 1;
      if (!(stop || q.k >= m || q.its >= p->o.max_outer)) continue;
      // end of the cycle: y = H^{-1} g, x += Z y, true residual
      const int nk = q.k;
      for (int i = nk - 1; i >= 0; --i) {
        double v = q.g[i];
        for (int j = i + 1; j < nk; ++j) v -= H[(size_t)i * m + j] * q.y[j];
        q.y[i] = v / H[(size_t)i * m + i];
      }
      const int ph2 = phase_open(p, s, PINTOC_PHASE_ORTH);
      HIPCHK(hipMemcpyAsync(p->dd, q.y.data(), sizeof(double) * nk, hipMemcpyHostToDevice, s));
      if (mb.Zk32)
        launch_lincomb_add_f32(s, x[k], mb.Zk32, n, nk, p->dd, n);
      else
        launch_lincomb_add(s, x[k], mb.Zk, n, nk, p->dd, n);
      phase_close(p, s, ph2);
      p->bytes_acc += ((mb.Zk32 ? 0.5 : 1.0) * nk + 2.0 + 4.0) * 8.0 * (double)n;
      kkt_t(p, x[k], mb.rvec, s, k);
      launch_axpby(s, mb.rvec, b[k], 1.0, -1.0, n);
      if ((rc = dots(p, s, mb.rvec, 1, mb.rvec, p->dd, hb, n))) return rc;
      q.res = std::sqrt(hb[0]);
      q.in_cycle = false;
      if ((q.breakdown || q.stalled) && !(q.res <= tol * q.bnorm)) q.done = true;
    }
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  bool all = true;
  for (const MemberSolve& q : ms) all &= q.conv;
  if (st) {
    double ph[PINTOC_NPHASES];
    phase_sum(p, ph);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < nm; ++k) {
      pintoc_solve_stats* o = &st[k];
      const MemberSolve& q = ms[k];
      const Member& mb = p->mem[k];
      double* hist_out = o->residual_history;
      const int hcap = o->history_capacity;
      int32_t* cnt_out = o->inner_counts;
      const int ccap = o->inner_counts_capacity;
      std::memset(o, 0, sizeof(*o));
      o->residual_history = hist_out;
      o->history_capacity = hcap;
      o->inner_counts = cnt_out;
      o->inner_counts_capacity = ccap;
      if (hist_out && hcap > 0) {
        o->history_length = (int32_t)std::min<size_t>((size_t)hcap, q.hist.size());
        std::copy(q.hist.begin(), q.hist.begin() + o->history_length, hist_out);
      }
      long isum = 0;
      for (int j = 0; j < mb.nf; ++j) {
        isum += p->its_acc[mb.f0 + j];
        if (cnt_out && j < ccap) cnt_out[j] = (int32_t)p->its_acc[mb.f0 + j];
      }
      for (int i = 0; i < PINTOC_NPHASES; ++i) o->phase_seconds[i] = ph[i];
      o->model_bytes = p->bytes_acc;                    // the whole group's
      o->precond_model_bytes = (p->model_fft + p->model_block) * mb.nf / p->nf;
      o->outer_iterations = q.its;
      o->converged = q.conv ? 1 : 0;
      o->rel_residual = q.bnorm > 0 ? q.res / q.bnorm : 0.0;
      o->precond_applications = q.apps;
      o->inner_iterations_mean = (p->o.inner != PINTOC_INNER_LINEAR && q.apps > 0) ? (double)isum / ((double)q.apps * mb.nf) : 0.0;
      o->inner_iterations_max = q.inner_max;
      o->seconds = secs;
    }
  }
  return all ? PINTOC_OK : PINTOC_NOT_CONVERGED;
}

extern "C" int pintoc_solve_batch(pintoc_problem* const* p, const double* const* b, double* const* x,
                                  pintoc_solve_stats* st, void* const* streams, int32_t n) {
  if (n < 0) return fail(PINTOC_EINVAL, "negative problem count");
  if (n == 0) return PINTOC_OK;
  if (!p || !b || !x || !streams) return fail(PINTOC_EINVAL, "NULL argument array");
  for (int k = 0; k < n; ++k) {
    if (!p[k] || !b[k] || !x[k] || !streams[k])
      return fail(PINTOC_EINVAL, "problem " + std::to_string(k) + ": NULL handle, vector or stream");
    if (!p[k]->bound) return fail(PINTOC_ESTATE, "problem " + std::to_string(k) + ": no workspace bound");
    for (int q = 0; q < k; ++q)
      if (p[q] == p[k] || streams[q] == streams[k])
        return fail(PINTOC_EINVAL, "problems " + std::to_string(q) + " and " + std::to_string(k) +
                                       " share a handle or a stream");
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::vector<int> rc(n, PINTOC_OK);
  std::vector<std::string> msg(n);
  std::vector<std::thread> th;
  th.reserve(n);
  for (int k = 0; k < n; ++k) {
    th.emplace_back([&, k]() {
      if (hipSetDevice(dev) != hipSuccess) {
        rc[k] = PINTOC_EHIP;
        msg[k] = "hipSetDevice failed in the worker thread";
        return;
      }
      rc[k] = pintoc_solve(p[k], b[k], x[k], st ? st + k : nullptr, streams[k]);
      if (rc[k] < 0) msg[k] = g_err;
    });
  }
  for (auto& t : th) t.join();
  int out = PINTOC_OK;
  for (int k = 0; k < n; ++k) {
    if (rc[k] < 0) return fail(rc[k], "problem " + std::to_string(k) + ": " + msg[k]);
    if (rc[k] == PINTOC_NOT_CONVERGED) out = PINTOC_NOT_CONVERGED;
  }
  return out;
}
