// Host runtime and C ABI: plan construction (FP64 constant tables, alpha
// choice), workspace layout, the outer iteration loop and the stage entry
// points.  Everything on the hot path runs in the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "pint.h"
#include "pint_kernels.hpp"
#include "pint_internal.hpp"

using namespace pint;

namespace {

thread_local std::string g_last_error;

int set_err(std::string* plan_err, int code, const std::string& msg) {
  g_last_error = msg;
  if (plan_err) *plan_err = msg;
  return code;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

struct pint_plan {
  pint_problem p;
  int dim, n, nt, ns;
  double h, alpha, a, dof, rtol;
  int max_iter;
  int nbl;          // row blocks per level (2D), 1 in 1D
  int nbl_f;        // blocks per level of the forward (residual) row pass
  int predict = 2;  // iterations enqueued before the first stop-flag check
  double safety = 0.1;
  bool fp64;   // working precision W = double
  bool mixed;  // FP64 forward spatial transform, FP32 time solve and inverse
  int dense = -1;  // DenseKind of the time contraction on the matrix cores, -1: FFT path
  bool norefine = false;  // residual and iterate in FP32 (no refinement)
  bool direct = false;    // nonuniform steps: direct diagonalization of the time-step pencil
  // The iteration may keep its spectral array in panels of a few time-solve
  // tiles (2D, FFT time path): each panel's N_t levels are contiguous for
  // the time solve; the column passes convert from / to the plain layout.
  bool tiled = false;
  int tps_spec = 0;   // log2 of the spectral panel width in the iteration
  int time_tile = 0;  // tuning cap on the time-solve tile (0: automatic)
  std::vector<double> dts;  // the steps (direct only)
  size_t off_dts = 0, off_idts = 0, off_v64 = 0, off_w64 = 0;  // direct tables in the block
  std::string err;

  // device tables (one allocation), FP64 then FP32 copies
  void* d_tab = nullptr;
  bool own_tab = true;
  size_t tab_bytes = 0;
  std::vector<unsigned char> host_tab;  // kept alive for asynchronous table copies
  size_t offs_d[11] = {}, offs_f[11] = {};  // table offsets (FP64 / FP32 copies) in the block
  size_t offs_w[4] = {};                     // dense W tables: F32 (wf, wb) or BF16 (wf hi/lo, wb hi/lo)
  DenseArgs dargs{};
  DctTables<double> dtd{};
  DctTables<float> dtf{};
  TimeArgs<double> tad{};
  TimeArgs<float> taf{};
  ResidArgs ra{};

  Ctrl* h_ctrl = nullptr;  // pinned host mirror written by the control kernel
  std::vector<hipEvent_t> ev;

  // solve graph (PINT_FLAG_SOLVE_GRAPH): init + the predicted iterations,
  // valid for the buffers, stream and iteration count it was captured with
  hipGraphExec_t gexec = nullptr;
  const void* g_u0 = nullptr;
  const void* g_U = nullptr;
  const void* g_work = nullptr;
  hipStream_t g_st = nullptr;
  int g_iters = 0;

  ~pint_plan() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (d_tab && own_tab) (void)hipFree(d_tab);
    if (h_ctrl) (void)hipHostFree(h_ctrl);
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

namespace {

struct HostTables {
  std::vector<std::complex<double>> tw_s, wq, wi, tw_t, lam1, pco, qco;
  std::vector<double> aj, aij, lamx, lamy;
};

double spectrum(int k, int n, double h) { return (2.0 / (h * h)) * (std::cos(M_PI * k / n) - 1.0); }

// Smallest eigenvalue of the spatial part of the preconditioned operator
// (A for the linear operators; Lap_h + eps^2 Lap_h^2 for CH with c_bar = 0).
// Every eigenvalue is mu(lam) = c1 lam + c2 lam^2 with c2 >= 0, lam = lx + ly
// a sum of 1D Laplacian eigenvalues.  mu is convex in lam, so for each lx the
// minimizing ly is one of the two neighbours of lam* - lx (lam* = -c1 / 2c2)
// in the sorted 1D spectrum: O(N log N) instead of a sweep over all N^2 modes.
double mu_min(const pint_problem& p, int dim, int n, double h) {
  double c1 = 0.0, c2 = 0.0;
  switch (p.op) {
    case PINT_OP_BIHARMONIC: c2 = 1.0; break;
    case PINT_OP_LINEAR_CH: c1 = p.beta * p.beta; c2 = p.eps * p.eps; break;
    case PINT_OP_CH: c1 = 1.0; c2 = p.eps * p.eps; break;
    default: c2 = p.eps * p.eps; break;  // Eyre: implicit part only
  }
  auto mu = [&](double lam) { return c1 * lam + c2 * lam * lam; };
  std::vector<double> lam(n);  // decreasing: lam[0] = 0 > lam[1] > ... > lam[n-1]
  for (int k = 0; k < n; ++k) lam[k] = spectrum(k, n, h);
  const double star = c2 > 0.0 ? -c1 / (2.0 * c2) : (c1 >= 0.0 ? -INFINITY : INFINITY);
  double best = 0.0;
  auto consider_row = [&](double lx) {
    const double target = star - lx;
    // first index whose eigenvalue is <= target (the array is decreasing)
    const auto it = std::lower_bound(lam.begin(), lam.end(), target, [](double a, double b) { return a > b; });
    const long j = long(it - lam.begin());
    for (long jj = j - 1; jj <= j; ++jj)
      if (jj >= 0 && jj < n) best = std::min(best, mu(lx + lam[size_t(jj)]));
  };
  if (dim == 2) {
    for (int kx = 0; kx < n; ++kx) consider_row(lam[kx]);
  } else {
    consider_row(0.0);
  }
  return best;
}

// Kind of dense time contraction a problem asks for (-1: the FFT path).
int dense_kind_of(const pint_problem* p) {
  if (p->dts) return p->precision == PINT_PREC_FP64 ? -1 : DK_F32;  // direct: FP32 MFMA or FP64 vector
  if (p->precision == PINT_PREC_BF16_REFINE || p->precision == PINT_PREC_BF16_NOREFINE)
    return (p->flags & PINT_FLAG_BF16_SPLIT) ? DK_BF16X3 : DK_BF16;
  if (p->time_path == PINT_TIME_DENSE) return DK_F32;
  return -1;
}

int validate(const pint_problem* p, std::string* err) {
  if (!p) return set_err(err, PINT_EINVAL, "problem is NULL");
  if (p->struct_size < sizeof(pint_problem)) return set_err(err, PINT_EINVAL, "pint_problem.struct_size too small");
  if (p->op < PINT_OP_BIHARMONIC || p->op > PINT_OP_CH_EYRE) return set_err(err, PINT_EINVAL, "unknown op");
  if (p->dim != 1 && p->dim != 2) return set_err(err, PINT_EINVAL, "dim must be 1 or 2");
  if (!is_pow2(p->nx) || p->nx < 8 || p->nx > 512)
    return set_err(err, PINT_EINVAL, "nx must be a power of two in [8, 512]");
  if (p->dim == 2 && p->ny != p->nx) return set_err(err, PINT_EINVAL, "2D grids must be square (ny == nx)");
  if (p->dim == 1 && p->ny != 1 && p->ny != 0) return set_err(err, PINT_EINVAL, "1D problems need ny == 1");
  if (!is_pow2(p->nt) || p->nt < 4 || p->nt > 1024)
    return set_err(err, PINT_EINVAL, "nt must be a power of two in [4, 1024]");
  if (!p->dts && (!(p->dt > 0.0) || !std::isfinite(p->dt))) return set_err(err, PINT_EINVAL, "dt must be > 0");
  if (p->dts) {
    // direct diagonalization of the time-step pencil (nonuniform steps)
    std::vector<double> st(p->dts, p->dts + p->nt);
    for (double x : st)
      if (!(x > 0.0) || !std::isfinite(x)) return set_err(err, PINT_EINVAL, "dts: every step must be > 0");
    std::sort(st.begin(), st.end());
    for (size_t i = 1; i < st.size(); ++i)
      if (!(st[i] - st[i - 1] > 1e-12 * st[i]))
        return set_err(err, PINT_EINVAL,
                       "dts: the steps must be pairwise distinct (equal steps make the time-step pencil "
                       "defective; use the uniform-step path)");
    if (p->op == PINT_OP_CH_EYRE)
      return set_err(err, PINT_EINVAL, "nonuniform steps: the Eyre scheme is not supported");
    if (p->precision != PINT_PREC_FP64 && p->precision != PINT_PREC_FP32_REFINE && p->precision != PINT_PREC_MIXED)
      return set_err(err, PINT_EINVAL, "nonuniform steps: precision must be FP64, FP32_REFINE or MIXED");
    if (p->time_path == PINT_TIME_FFT)
      return set_err(err, PINT_EINVAL, "nonuniform steps: the time solve is the direct contraction, not the FFT");
    if (p->nt < 32) return set_err(err, PINT_EINVAL, "nonuniform steps need nt >= 32");
    const int ns = p->dim == 2 ? p->nx * p->nx : p->nx;
    if (ns % dense_cols_per_block(p->nt) != 0 || ns % 32 != 0)
      return set_err(err, PINT_EINVAL, "nonuniform steps: N_s must be a multiple of " +
                                           std::to_string(std::max(32, dense_cols_per_block(p->nt))));
  }
  const bool linear = p->op == PINT_OP_BIHARMONIC || p->op == PINT_OP_LINEAR_CH;
  if (linear && !(p->theta == 1.0 || p->theta == 0.5)) return set_err(err, PINT_EINVAL, "theta must be 1 or 0.5");
  if (!linear && p->theta != 1.0 && p->theta != 0.0)
    return set_err(err, PINT_EINVAL, "the CH schemes are backward Euler (theta = 1)");
  if (p->op != PINT_OP_BIHARMONIC && !(p->eps > 0.0)) return set_err(err, PINT_EINVAL, "eps must be > 0");
  if (!p->dts && !(p->alpha >= 0.0 && p->alpha < 1.0))
    return set_err(err, PINT_EINVAL, "alpha must be in (0, 1) (0 = auto)");
  if (p->precision != PINT_PREC_FP64 && p->precision != PINT_PREC_FP32_REFINE && p->precision != PINT_PREC_MIXED &&
      p->precision != PINT_PREC_BF16_REFINE && p->precision != PINT_PREC_FP32_NOREFINE &&
      p->precision != PINT_PREC_BF16_NOREFINE)
    return set_err(err, PINT_EINVAL, "precision not supported by this build");
  if (p->precision == PINT_PREC_FP32_NOREFINE && p->time_path == PINT_TIME_DENSE)
    return set_err(err, PINT_EINVAL, "the unrefined mode uses the FFT time path");
  if (p->time_path != PINT_TIME_AUTO && p->time_path != PINT_TIME_FFT && p->time_path != PINT_TIME_DENSE)
    return set_err(err, PINT_EINVAL, "unknown time path");
  if (p->precision == PINT_PREC_FP64 && p->time_path == PINT_TIME_DENSE)
    return set_err(err, PINT_EINVAL, "the dense time contraction computes in FP32 or BF16, not FP64");
  if ((p->precision == PINT_PREC_BF16_REFINE || p->precision == PINT_PREC_BF16_NOREFINE) &&
      p->time_path == PINT_TIME_FFT)
    return set_err(err, PINT_EINVAL, "BF16 is a precision of the dense time contraction, not of the FFT path");
  if (dense_kind_of(p) >= 0 && !p->dts) {
    const int nb = dense_cols_per_block(p->nt);
    const int ns = p->dim == 2 ? p->nx * p->nx : p->nx;
    if (nb == 0 || ns % nb != 0)
      return set_err(err, PINT_EINVAL, "the dense time contraction needs N_t >= 32 and N_s a multiple of " +
                                           std::to_string(nb ? nb : 32));
  }
  if (p->flags & PINT_FLAG_FIELD_JACOBIAN) {
    if (p->op != PINT_OP_CH)
      return set_err(err, PINT_EINVAL, "the space-varying averaged Jacobian is for the PinT-I CH operator");
    if (p->precision == PINT_PREC_FP32_NOREFINE || p->precision == PINT_PREC_BF16_NOREFINE)
      return set_err(err, PINT_EINVAL, "the space-varying averaged Jacobian needs a refined precision");
    if (p->flags & (PINT_FLAG_SOLVE_GRAPH | PINT_FLAG_STAGE_TIMING))
      return set_err(err, PINT_EINVAL, "the space-varying averaged Jacobian takes no solve graph or stage timing");
  }
  if (p->max_iter < 0 || p->max_iter > PINT_HIST) return set_err(err, PINT_EINVAL, "max_iter must be in [0, 64]");
  if (p->rtol < 0.0) return set_err(err, PINT_EINVAL, "rtol must be >= 0");
  const double lx = p->lx > 0 ? p->lx : 1.0;
  if (!std::isfinite(lx)) return set_err(err, PINT_EINVAL, "lx must be finite");
  return PINT_OK;
}

void build_tables(pint_plan* pl, HostTables& t) {
  const int n = pl->n, nt = pl->nt;
  const double h = pl->h, dt = pl->p.dt, a = pl->a, th = pl->p.theta;
  const double la = pl->direct ? 0.0 : std::log(pl->alpha) / nt;  // log a (no alpha for direct)
  t.tw_s.resize(n);
  t.wq.resize(n);
  t.wi.resize(n);
  for (int m = 0; m < n; ++m) {
    const double ang = -2.0 * M_PI * m / n;
    t.tw_s[m] = {std::cos(ang), std::sin(ang)};
    const double s = m == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
    const double q = M_PI * m / (2.0 * n);
    t.wq[m] = s * std::complex<double>(std::cos(q), -std::sin(q));
    t.wi[m] = std::complex<double>(std::cos(q), std::sin(q)) / s;
  }
  t.tw_t.resize(nt);
  t.lam1.resize(nt);
  t.pco.resize(nt);
  t.qco.resize(nt);
  t.aj.resize(nt);
  t.aij.resize(nt);
  const double e2 = pl->p.eps * pl->p.eps, b2 = pl->p.beta * pl->p.beta;
  for (int l = 0; l < nt; ++l) {
    const double ang = -2.0 * M_PI * l / nt;
    const std::complex<double> w(std::cos(ang), std::sin(ang));
    t.tw_t[l] = w;
    // Time eigenvalues of the alpha-circulant blocks (Lemma of Section 2.1)
    // in the exp(-2 pi i l / N_t) ordering of the forward FFT.
    t.lam1[l] = (1.0 - a * w) / dt;
    const std::complex<double> lam2 = th + (1.0 - th) * a * w;
    switch (pl->p.op) {
      case PINT_OP_BIHARMONIC:
        t.pco[l] = 0.0;
        t.qco[l] = lam2;
        break;
      case PINT_OP_LINEAR_CH:
        t.pco[l] = b2 * lam2;
        t.qco[l] = e2 * lam2;
        break;
      case PINT_OP_CH:  // lambda1 + (1 - c_bar) lam + eps^2 lam^2 (eq. pintiter_CH)
        t.pco[l] = 1.0;
        t.qco[l] = e2;
        break;
      default:  // Eyre: lambda1 + (lambda3 - c_bar) lam + eps^2 lam^2 (eq. pintiter_CH_eyre)
        t.pco[l] = a * w;
        t.qco[l] = e2;
        break;
    }
    if (pl->direct) {
      // direct diagonalization: row j of the contraction is eigen-coordinate
      // j, divided by d_j + p lam + q lam^2 with d_j = 1/(theta dt_j) from the
      // GPU eigendecomposition (lam1 is filled there) and the operator's
      // spatial coefficients (the theta of the pencil sits in d_j and C)
      t.lam1[l] = 0.0;
      switch (pl->p.op) {
        case PINT_OP_BIHARMONIC: t.pco[l] = 0.0; t.qco[l] = 1.0; break;
        case PINT_OP_LINEAR_CH: t.pco[l] = b2; t.qco[l] = e2; break;
        default: t.pco[l] = 1.0; t.qco[l] = e2; break;  // CH: (1 - c_bar) lam + eps^2 lam^2
      }
    }
    t.aj[l] = std::exp(la * l);
    t.aij[l] = std::exp(-la * l) / nt;
  }
  t.lamx.resize(n);
  for (int k = 0; k < n; ++k) t.lamx[k] = spectrum(k, n, h);
  if (pl->dim == 2) {
    t.lamy = t.lamx;
  } else {
    t.lamy.assign(1, 0.0);
  }
}

template <typename T>
size_t put_cx(std::vector<unsigned char>& buf, size_t off, const std::vector<std::complex<double>>& v) {
  off = align256(off);
  buf.resize(off + v.size() * 2 * sizeof(T));
  T* d = reinterpret_cast<T*>(buf.data() + off);
  for (size_t i = 0; i < v.size(); ++i) {
    d[2 * i] = T(v[i].real());
    d[2 * i + 1] = T(v[i].imag());
  }
  return off;
}
template <typename T>
size_t put_re(std::vector<unsigned char>& buf, size_t off, const std::vector<double>& v) {
  off = align256(off);
  buf.resize(off + v.size() * sizeof(T));
  T* d = reinterpret_cast<T*>(buf.data() + off);
  for (size_t i = 0; i < v.size(); ++i) d[i] = T(v[i]);
  return off;
}

struct Offs {
  size_t tw_s, wq, wi, tw_t, lam1, pco, qco, aj, aij, lamx, lamy;
};

template <typename T>
Offs put_all(std::vector<unsigned char>& buf, const HostTables& t) {
  Offs o;
  o.tw_s = put_cx<T>(buf, buf.size(), t.tw_s);
  o.wq = put_cx<T>(buf, buf.size(), t.wq);
  o.wi = put_cx<T>(buf, buf.size(), t.wi);
  o.tw_t = put_cx<T>(buf, buf.size(), t.tw_t);
  o.lam1 = put_cx<T>(buf, buf.size(), t.lam1);
  o.pco = put_cx<T>(buf, buf.size(), t.pco);
  o.qco = put_cx<T>(buf, buf.size(), t.qco);
  o.aj = put_re<T>(buf, buf.size(), t.aj);
  o.aij = put_re<T>(buf, buf.size(), t.aij);
  o.lamx = put_re<T>(buf, buf.size(), t.lamx);
  o.lamy = put_re<T>(buf, buf.size(), t.lamy);
  return o;
}

// Space for the dense time-contraction matrices (each N_t x N_t, 256-byte
// aligned): DK_F32 two FP32 arrays, the BF16 kinds four BF16 arrays.
void reserve_dense(std::vector<unsigned char>& buf, int kind, int nt, size_t* offs) {
  if (kind < 0) return;
  const size_t bytes = size_t(nt) * nt * (kind == DK_F32 ? 4 : 2);
  const int count = kind == DK_F32 ? 2 : 4;
  for (int i = 0; i < count; ++i) {
    offs[i] = align256(buf.size());
    buf.resize(offs[i] + bytes);
  }
}

uint16_t bf16_round(float f) {  // round to nearest even (finite values)
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
float bf16_value(uint16_t h) {
  const uint32_t u = uint32_t(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// The dense forward and inverse time matrices of one spatial mode (FP64):
//   W_f[r][n] = a^n {1, (-1)^n, cos(2 pi l n/N_t), -sin(2 pi l n/N_t)}        r = 0, 1, 2l, 2l+1
//   W_b[n][r] = a^{-n}/N_t {1, (-1)^n, 2 cos(2 pi l n/N_t), -2 sin(2 pi l n/N_t)}
// so that W_b diag-divide W_f is Gamma^{-1} F^{-1} D^{-1} F Gamma on real data
// (Section 2.1, eq. pintiter1), with the Hermitian half-spectrum packed into
// N_t real rows.  Stored as FP32 transposes (DK_F32) or BF16 hi/lo row-major.
void put_dense(std::vector<unsigned char>& buf, const pint_plan* pl, const size_t* offs) {
  const int nt = pl->nt;
  const double la = std::log(pl->alpha) / nt;
  std::vector<double> wf(size_t(nt) * nt), wb(size_t(nt) * nt);
  for (int r = 0; r < nt; ++r) {
    const int l = r >> 1;
    for (int n = 0; n < nt; ++n) {
      const double an = std::exp(la * n), ain = std::exp(-la * n) / nt;
      const double ang = 2.0 * M_PI * double((long(l) * n) % nt) / nt;
      const double sgn = (n & 1) ? -1.0 : 1.0;
      double f, b;
      if (r == 0) {
        f = an;
        b = ain;
      } else if (r == 1) {
        f = an * sgn;
        b = ain * sgn;
      } else if ((r & 1) == 0) {
        f = an * std::cos(ang);
        b = 2.0 * ain * std::cos(ang);
      } else {
        f = -an * std::sin(ang);
        b = -2.0 * ain * std::sin(ang);
      }
      wf[size_t(r) * nt + n] = f;  // W_f[r][n]
      wb[size_t(n) * nt + r] = b;  // W_b[n][r]
    }
  }
  if (pl->dense == DK_F32) {
    float* tf = reinterpret_cast<float*>(buf.data() + offs[0]);
    float* tb = reinterpret_cast<float*>(buf.data() + offs[1]);
    for (int m = 0; m < nt; ++m)
      for (int k = 0; k < nt; ++k) {
        tf[size_t(k) * nt + m] = float(wf[size_t(m) * nt + k]);
        tb[size_t(k) * nt + m] = float(wb[size_t(m) * nt + k]);
      }
    return;
  }
  const std::vector<double>* src[2] = {&wf, &wb};
  for (int w = 0; w < 2; ++w) {
    uint16_t* hi = reinterpret_cast<uint16_t*>(buf.data() + offs[2 * w]);
    uint16_t* lo = reinterpret_cast<uint16_t*>(buf.data() + offs[2 * w + 1]);
    for (size_t i = 0; i < size_t(nt) * nt; ++i) {
      const double v = (*src[w])[i];
      hi[i] = bf16_round(float(v));
      lo[i] = bf16_round(float(v - double(bf16_value(hi[i]))));
    }
  }
}

// Direct diagonalization: the steps and 1/dt_n (FP64, for the residual) and
// room for the FP64 eigenvector matrices V [n][j] and W [j][n], which the GPU
// computes (k_eig_steps) after the upload.
void reserve_direct(std::vector<unsigned char>& buf, pint_plan* pl) {
  const int nt = pl->nt;
  std::vector<double> idts(nt);
  for (int i = 0; i < nt; ++i) idts[i] = 1.0 / pl->dts[i];
  pl->off_dts = put_re<double>(buf, buf.size(), pl->dts);
  pl->off_idts = put_re<double>(buf, buf.size(), idts);
  pl->off_v64 = align256(buf.size());
  buf.resize(pl->off_v64 + size_t(nt) * nt * 8);
  pl->off_w64 = align256(buf.size());
  buf.resize(pl->off_w64 + size_t(nt) * nt * 8);
}

void store_offs(const Offs& o, size_t* dst) {
  const size_t v[11] = {o.tw_s, o.wq, o.wi, o.tw_t, o.lam1, o.pco, o.qco, o.aj, o.aij, o.lamx, o.lamy};
  for (int i = 0; i < 11; ++i) dst[i] = v[i];
}
Offs load_offs(const size_t* s) { return Offs{s[0], s[1], s[2], s[3], s[4], s[5], s[6], s[7], s[8], s[9], s[10]}; }

template <typename T>
void bind(const Offs& o, unsigned char* base, const pint_plan* pl, DctTables<T>& dt, TimeArgs<T>& ta) {
  dt.tw = reinterpret_cast<const cx<T>*>(base + o.tw_s);
  dt.wq = reinterpret_cast<const cx<T>*>(base + o.wq);
  dt.wi = reinterpret_cast<const cx<T>*>(base + o.wi);
  ta.tw = reinterpret_cast<const cx<T>*>(base + o.tw_t);
  ta.lam1 = reinterpret_cast<const cx<T>*>(base + o.lam1);
  ta.pco = reinterpret_cast<const cx<T>*>(base + o.pco);
  ta.qco = reinterpret_cast<const cx<T>*>(base + o.qco);
  ta.aj = reinterpret_cast<const T*>(base + o.aj);
  ta.aij = reinterpret_cast<const T*>(base + o.aij);
  ta.lamx = reinterpret_cast<const T*>(base + o.lamx);
  ta.lamy = reinterpret_cast<const T*>(base + o.lamy);
  ta.nx = pl->n;
  ta.ns = pl->ns;
  ta.cbar_mode = (pl->p.op == PINT_OP_CH || pl->p.op == PINT_OP_CH_EYRE) ? 1 : 0;
  ta.cbar = nullptr;
  ta.done = nullptr;
  ta.tile = pl->time_tile;
  ta.tps = ilog2(pl->ns);
  ta.bcast_in = 0;
}

struct Work {
  void* S;    // spectral scratch in the working type W
  void* S64;  // FP64 forward-transform scratch (mixed precision only)
  void* ST;   // tiled spectral array in W (tiled plans only)
  double* part;
  double* fin;  // first-stage results of the two-stage control reduction
  Ctrl* ctrl;
};

// Partial-result slots: one per [level][row block]; the initial c_bar
// reduction needs one per 4096 values of the initial guess.
size_t part_bytes(const pint_plan* pl) {
  const size_t slots = std::max<size_t>((size_t)pl->nt * std::max(pl->nbl, pl->nbl_f),
                                        ((size_t)pl->nt * pl->ns + 4095) / 4096);
  return align256(slots * PART_STRIDE * 8);
}
size_t s_bytes(const pint_plan* pl) { return align256((size_t)pl->nt * pl->ns * (pl->fp64 ? 8 : 4)); }
size_t s64_bytes(const pint_plan* pl) { return pl->mixed ? align256((size_t)pl->nt * pl->ns * 8) : 0; }
size_t st_bytes(const pint_plan* pl) { return pl->tiled ? s_bytes(pl) : 0; }

size_t fin_bytes(const pint_plan* pl) {
  return align256(size_t(std::max(1, finalize_groups(pl->nt, pl->nbl, pl->nbl_f))) * 4 * sizeof(double));
}
// Inner solve of the space-varying averaged Jacobian (PINT_FLAG_FIELD_JACOBIAN):
// eight FP64 space-time vectors, the field, dot-product partials and the
// operator's own residual partials.
constexpr int FIELD_VECS = 8;
bool field_mode(const pint_plan* pl) { return (pl->p.flags & PINT_FLAG_FIELD_JACOBIAN) != 0; }
size_t field_bytes(const pint_plan* pl) {
  if (!field_mode(pl)) return 0;
  return FIELD_VECS * align256(size_t(pl->nt) * pl->ns * 8) + align256(size_t(pl->ns) * 8) +
         align256(size_t(4) * DOT_BLOCKS * 8) + part_bytes(pl);
}
size_t work_size(const pint_plan* pl) {
  return s_bytes(pl) + s64_bytes(pl) + st_bytes(pl) + part_bytes(pl) + fin_bytes(pl) + align256(sizeof(Ctrl)) +
         field_bytes(pl);
}

int carve(pint_plan* pl, void* d_work, size_t bytes, Work& w) {
  if (!d_work) return set_err(&pl->err, PINT_EINVAL, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return set_err(&pl->err, PINT_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < work_size(pl)) return set_err(&pl->err, PINT_ENOMEM, "workspace smaller than pint_plan_workspace_size");
  unsigned char* b = static_cast<unsigned char*>(d_work);
  w.S = b;
  b += s_bytes(pl);
  w.S64 = pl->mixed ? b : nullptr;
  b += s64_bytes(pl);
  w.ST = st_bytes(pl) ? b : nullptr;
  b += st_bytes(pl);
  w.part = reinterpret_cast<double*>(b);
  b += part_bytes(pl);
  w.fin = reinterpret_cast<double*>(b);
  b += fin_bytes(pl);
  w.ctrl = reinterpret_cast<Ctrl*>(b);
  return PINT_OK;
}

int hip_fail(pint_plan* pl, hipError_t e, const char* what) {
  return set_err(pl ? &pl->err : nullptr, PINT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr, what)                          \
  do {                                              \
    hipError_t e__ = (expr);                        \
    if (e__ != hipSuccess) return hip_fail(pl, e__, what); \
  } while (0)

constexpr int EV_PER_IT = 12;  // a (start, stop) event pair for each of the 6 kernels of one iteration

template <typename T>
const DctTables<T>& dct_tables(const pint_plan* pl);
template <>
const DctTables<double>& dct_tables<double>(const pint_plan* pl) { return pl->dtd; }
template <>
const DctTables<float>& dct_tables<float>(const pint_plan* pl) { return pl->dtf; }
template <typename T>
TimeArgs<T> time_args(const pint_plan* pl);
template <>
TimeArgs<double> time_args<double>(const pint_plan* pl) { return pl->tad; }
template <>
TimeArgs<float> time_args<float>(const pint_plan* pl) { return pl->taf; }

// Enqueue one outer iteration: row pass (residual + x-DCT), column pass
// (y-DCT), time solve, column pass (y-DCT-III), row pass (x-DCT-III + update),
// control.  TF is the type of the forward spatial transform, T that of the
// time solve and the inverse transform.  bcast: the iterate is the broadcast
// datum u0 (first iteration).
// a3-a5 on the plan's time path: the FFT kernel, or the dense contraction on
// the matrix cores (FP32 working type only).
template <typename T>
hipError_t launch_time_any(const pint_plan* pl, T* S, const TimeArgs<T>& ta, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (pl->dense >= 0) return launch_time_dense(pl->dense, pl->nt, S, ta, pl->dargs, st);
  } else {
    if (pl->direct) return launch_time_direct64(pl->nt, S, ta, pl->dargs, st);
  }
  return launch_time<T>(pl->nt, S, ta, st);
}

template <typename TF, typename T, typename RT = double>
int enqueue_iteration(pint_plan* pl, const double* d_u0, double* d_U, const Work& w, hipStream_t st,
                      hipEvent_t* evs, bool bcast, Ctrl* host) {
  TimeArgs<T> ta = time_args<T>(pl);
  ta.cbar = &w.ctrl->c_bar;
  ta.done = &w.ctrl->done;
  ResidArgs ra = pl->ra;
  ra.u0 = d_u0;
  ra.U = d_U;
  ra.part = w.part;
  ra.done = &w.ctrl->done;
  ra.bcast = bcast ? 1 : 0;
  // First sweep from the broadcast datum (2D, FFT time path): every level's
  // residual and spatial transform are level 0's, so the row and column
  // passes run on level 0 and the time solve reads it for every level.
  const bool one = bcast && pl->dim == 2 && pl->dense < 0 && !pl->direct;
  ra.one_level = one ? 1 : 0;
  if (one) ra.nt = pl->nt;
  ta.bcast_in = one ? 1 : 0;
  FinArgs fa{w.ctrl, host, w.part, w.fin, pl->nt, pl->nbl, pl->max_iter, pl->nbl_f, pl->norefine ? 1 : 0,
             pl->dof, pl->rtol, pl->safety};
  UpdArgs ua{d_U, d_u0, w.part, &w.ctrl->done, bcast ? 1 : 0, pl->norefine ? 1 : 0};
  T* S = static_cast<T*>(w.S);
  TF* SF = std::is_same<TF, T>::value ? reinterpret_cast<TF*>(w.S) : static_cast<TF*>(w.S64);
  const int* done = &w.ctrl->done;
  // SP: the spectral array of the time solve, tiled in ST or plain in S (the
  // column passes then work in place); the inverse row pass reads plain S.
  T* SP = S;
  const int tpn = ilog2(pl->ns);
  if (pl->tiled) {
    SP = static_cast<T*>(w.ST);
    ta.tps = pl->tps_spec;
  }
  // stage timing: each kernel is bracketed by its own (start, stop) event pair
  auto ev = [&](int stage) {
    if (evs) set_launch_events(evs[2 * stage], evs[2 * stage + 1]);
  };
  ev(0);
  if (pl->dim == 2)
    HIPCHK((launch_rows_fwd<TF, TF, RT>(2, pl->n, ra, SF, nullptr, dct_tables<TF>(pl), pl->nt, 0, st)),
           "residual + x-DCT kernel");
  else
    HIPCHK((launch_rows_fwd<TF, T, RT>(1, pl->n, ra, S, nullptr, dct_tables<TF>(pl), pl->nt, 0, st)),
           "residual + x-DCT kernel");
  if (pl->dim == 2) {
    ev(1);
    HIPCHK((launch_cols<TF, T>(pl->n, SF, SP, done, dct_tables<TF>(pl), pl->nt, false, st, tpn, ta.tps,
                               one ? 1 : pl->nt)),
           "y-DCT kernel");
  }
  ev(2);
  HIPCHK(launch_time_any<T>(pl, SP, ta, st), "time-solve kernel");
  if (pl->dim == 2) {
    ev(3);
    HIPCHK((launch_cols<T, T>(pl->n, SP, S, done, dct_tables<T>(pl), pl->nt, true, st, ta.tps, tpn)),
           "y-DCT-III kernel");
  }
  ev(4);
  HIPCHK(launch_rows_inv<T>(pl->dim, pl->n, ua, S, nullptr, dct_tables<T>(pl), pl->nt, 0, st),
         "x-DCT-III + update kernel");
  ev(5);
  HIPCHK(launch_finalize(fa, st), "control kernel");
  set_launch_events(nullptr, nullptr);
  return PINT_OK;
}

int enqueue_any(pint_plan* pl, const double* d_u0, double* d_U, const Work& w, hipStream_t st, hipEvent_t* evs,
                bool bcast, Ctrl* host) {
  if (pl->fp64) return enqueue_iteration<double, double>(pl, d_u0, d_U, w, st, evs, bcast, host);
  if (pl->mixed) return enqueue_iteration<double, float>(pl, d_u0, d_U, w, st, evs, bcast, host);
  if (pl->norefine) return enqueue_iteration<float, float, float>(pl, d_u0, d_U, w, st, evs, bcast, host);
  return enqueue_iteration<float, float>(pl, d_u0, d_U, w, st, evs, bcast, host);
}

int begin_solve(pint_plan* pl, const double* d_u0, double* d_U, const Work& w, hipStream_t st, Ctrl* host) {
  const bool bcast = (pl->p.flags & PINT_FLAG_INIT_BROADCAST_U0) != 0;
  InitArgs ia{d_u0, d_U, w.part, pl->nt, pl->ns, pl->nbl, bcast ? 1 : 0};
  const bool need_cbar = pl->p.op == PINT_OP_CH || pl->p.op == PINT_OP_CH_EYRE;
  HIPCHK(launch_init(ia, w.ctrl, host, pl->dof, need_cbar, st), "init kernels");
  return PINT_OK;
}

// ---------------------------------------------------------------------------
// Outer iteration with the space-varying averaged Jacobian (eq. approx_jacobian,
// PinT-I): U <- U + G~'(U)^{-1} r(U), with
//   G~'(U) = C1^(alpha) (x) I - I (x) Lap_h J~ + I (x) Lap_h + eps^2 I (x) Lap_h^2,
//   J~ = diag((1/N_t) sum_n 3 u_n^2),
// whose Step-(2) systems are not diagonal in the cosine basis.  The linear
// system is solved by BiCGStab on the space-time vectors, right-
// preconditioned by the scalar-c_bar solve (the plan's own preconditioner:
// DCT, alpha-circulant time solve, inverse DCT), until the inner residual has
// dropped by FIELD_INNER_RTOL or FIELD_INNER_MAX iterations.  The operator is
// applied in physical space by the residual kernel with the field in place
// of the cubic term and the alpha corner in place of u0.  Every scalar of the
// iteration comes from fixed-order reductions, so the solve is deterministic.
constexpr double FIELD_INNER_RTOL = 1e-3;
constexpr int FIELD_INNER_MAX = 30;

struct FieldWork {
  double* v[FIELD_VECS];  // R, X, Rh, P, Vn, Tn, Ph, Sh
  double* jfield;
  double* dots;           // [4][DOT_BLOCKS]
  double* apart;          // partials of the operator applications
};

int field_carve(pint_plan* pl, void* d_work, FieldWork& f) {
  unsigned char* b = static_cast<unsigned char*>(d_work) + (work_size(pl) - field_bytes(pl));
  const size_t vb = align256(size_t(pl->nt) * pl->ns * 8);
  for (int i = 0; i < FIELD_VECS; ++i, b += vb) f.v[i] = reinterpret_cast<double*>(b);
  f.jfield = reinterpret_cast<double*>(b);
  b += align256(size_t(pl->ns) * 8);
  f.dots = reinterpret_cast<double*>(b);
  b += align256(size_t(4) * DOT_BLOCKS * 8);
  f.apart = reinterpret_cast<double*>(b);
  return PINT_OK;
}

// Pinned host buffer for the dot-product partials of one solve.
struct PinnedDots {
  double* p = nullptr;
  ~PinnedDots() {
    if (p) (void)hipHostFree(p);
  }
};

// Solve G~'(U) X = R (R is overwritten) with the field f.jfield of U already
// computed; cbar is the scalar averaged Jacobian of the preconditioner.
int field_inner_solve(pint_plan* pl, const double* d_u0, FieldWork& f, double* R, double* X, double cbar,
                      double rtol, int maxit, void* d_work, size_t work_bytes, hipStream_t st, double* hdots,
                      int* iters) {
  double *Rh = f.v[2], *P = f.v[3], *Vn = f.v[4], *Tn = f.v[5], *Ph = f.v[6], *Sh = f.v[7];
  const size_t n = size_t(pl->nt) * pl->ns;
  int rc = PINT_OK;
  auto dots = [&](std::initializer_list<std::pair<const double*, const double*>> prs, double* out) -> int {
    const double* xs[4];
    const double* ys[4];
    int q = 0;
    for (auto& pr : prs) {
      xs[q] = pr.first;
      ys[q] = pr.second;
      ++q;
    }
    HIPCHK(launch_dots(xs, ys, q, n, f.dots, st), "dot kernel");
    HIPCHK(hipMemcpyAsync(hdots, f.dots, size_t(q) * DOT_BLOCKS * sizeof(double), hipMemcpyDeviceToHost, st),
           "dot copy");
    HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
    for (int k = 0; k < q; ++k) {
      double acc = 0.0;
      for (int b = 0; b < DOT_BLOCKS; ++b) acc += hdots[size_t(k) * DOT_BLOCKS + b];
      out[k] = acc;
    }
    return PINT_OK;
  };
  // out = -G~' v (the residual kernel with b = 0)
  auto apply_neg = [&](const double* v, double* out) -> int {
    ResidArgs ra = pl->ra;
    ra.u0 = d_u0;  // not read: the first level's predecessor is the alpha corner
    ra.U = v;
    ra.part = f.apart;
    ra.done = nullptr;
    ra.bcast = 0;
    ra.jfield = f.jfield;
    ra.wrap = 1;
    ra.nt = pl->nt;
    ra.wrap_alpha = pl->alpha;
    HIPCHK((launch_rows_fwd<double, double, double>(pl->dim, pl->n, ra, nullptr, out, pl->dtd, pl->nt, 1, st)),
           "operator kernel");
    return PINT_OK;
  };
  auto axpy = [&](double* out, double a, const double* x, double b, const double* y, double c,
                  const double* z) -> int {
    HIPCHK(launch_axpbypcz(out, a, x, b, y, c, z, n, st), "vector kernel");
    return PINT_OK;
  };
  auto M = [&](const double* in, double* out) {
    return pint_precond_apply(pl, in, out, cbar, d_work, work_bytes, st);
  };
  *iters = 0;
  double d2[4];
  if ((rc = dots({{R, R}}, d2))) return rc;
  const double bnorm = std::sqrt(d2[0]);
  if ((rc = M(R, X))) return rc;                       // x0 = M r (the scalar-c_bar step)
  if ((rc = apply_neg(X, Tn))) return rc;              // r0 = r - A x0 = r + Tn
  if ((rc = axpy(R, 1.0, R, 1.0, Tn, 0.0, nullptr))) return rc;
  if ((rc = axpy(Rh, 1.0, R, 0.0, R, 0.0, nullptr))) return rc;
  HIPCHK(hipMemsetAsync(P, 0, n * sizeof(double), st), "hipMemsetAsync");
  HIPCHK(hipMemsetAsync(Vn, 0, n * sizeof(double), st), "hipMemsetAsync");
  double rho = 1.0, alpha = 1.0, omega = 1.0;
  if ((rc = dots({{Rh, R}, {R, R}}, d2))) return rc;
  double rho_new = d2[0], rnorm = std::sqrt(d2[1]);
  for (int in = 0; in < maxit && rnorm > rtol * bnorm && rho_new != 0.0; ++in) {
    ++*iters;
    const double beta = (rho_new / rho) * (alpha / omega);
    // p = r + beta (p - omega v), with v = -Vn
    if ((rc = axpy(P, 1.0, R, beta, P, beta * omega, Vn))) return rc;
    if ((rc = M(P, Ph))) return rc;
    if ((rc = apply_neg(Ph, Vn))) return rc;           // v = A ph = -Vn
    if ((rc = dots({{Rh, Vn}}, d2))) return rc;
    alpha = -rho_new / d2[0];
    if ((rc = axpy(R, 1.0, R, alpha, Vn, 0.0, nullptr))) return rc;  // s = r - alpha v (in R)
    if ((rc = M(R, Sh))) return rc;
    if ((rc = apply_neg(Sh, Tn))) return rc;           // t = A sh = -Tn
    if ((rc = dots({{Tn, R}, {Tn, Tn}}, d2))) return rc;
    omega = d2[1] > 0.0 ? -d2[0] / d2[1] : 0.0;        // (t, s) / (t, t)
    if ((rc = axpy(X, 1.0, X, alpha, Ph, omega, Sh))) return rc;
    if ((rc = axpy(R, 1.0, R, omega, Tn, 0.0, nullptr))) return rc;  // r = s - omega t
    rho = rho_new;
    if ((rc = dots({{Rh, R}, {R, R}}, d2))) return rc;
    rho_new = d2[0];
    rnorm = std::sqrt(d2[1]);
    if (omega == 0.0) break;
  }
  return PINT_OK;
}

int solve_field(pint_plan* pl, const double* d_u0, double* d_U, void* d_work, size_t work_bytes, const Work& w,
                hipStream_t st, int* inner_total) {
  FieldWork f;
  field_carve(pl, d_work, f);
  double *R = f.v[0], *X = f.v[1];
  const size_t n = size_t(pl->nt) * pl->ns;
  PinnedDots hd;
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hd.p), 4 * DOT_BLOCKS * sizeof(double), hipHostMallocDefault),
         "hipHostMalloc(dot partials)");
  const bool bcast = (pl->p.flags & PINT_FLAG_INIT_BROADCAST_U0) != 0;
  if (bcast) {
    HIPCHK(hipMemsetAsync(X, 0, n * sizeof(double), st), "hipMemsetAsync");
    HIPCHK(launch_update_plain(d_U, d_u0, X, w.part, pl->nt, pl->ns, pl->nbl, 1, st), "broadcast");
  }
  InitArgs ia{d_u0, d_U, w.part, pl->nt, pl->ns, pl->nbl, 0};
  HIPCHK(launch_init(ia, w.ctrl, pl->h_ctrl, pl->dof, true, st), "init kernels");
  FinArgs fa{w.ctrl, pl->h_ctrl, w.part, w.fin, pl->nt, pl->nbl, pl->max_iter, pl->nbl_f, 0, pl->dof, pl->rtol,
             pl->safety};
  *inner_total = 0;
  for (int it = 0; it < pl->max_iter; ++it) {
    // outer residual r(U) (FP64, alpha = 0) and the field of U
    ResidArgs ra = pl->ra;
    ra.u0 = d_u0;
    ra.U = d_U;
    ra.part = w.part;
    ra.done = nullptr;
    ra.bcast = 0;
    HIPCHK((launch_rows_fwd<double, double, double>(pl->dim, pl->n, ra, nullptr, R, pl->dtd, pl->nt, 1, st)),
           "residual kernel");
    HIPCHK(launch_jfield(d_U, f.jfield, pl->nt, pl->ns, st), "field kernel");
    HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
    const double cbar = reinterpret_cast<volatile double&>(pl->h_ctrl->c_bar);
    int iters = 0;
    const int rc = field_inner_solve(pl, d_u0, f, R, X, cbar, FIELD_INNER_RTOL, FIELD_INNER_MAX, d_work, work_bytes,
                                     st, hd.p, &iters);
    if (rc) return rc;
    *inner_total += iters;
    // U += delta, partials, control (stop rule, next c_bar)
    HIPCHK(launch_update_plain(d_U, d_u0, X, w.part, pl->nt, pl->ns, pl->nbl, 0, st), "update kernel");
    HIPCHK(launch_finalize(fa, st), "control kernel");
    HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (reinterpret_cast<volatile int&>(pl->h_ctrl->done)) break;
  }
  return PINT_OK;
}

void fill_report(const pint_plan* pl, const Ctrl& c, int status, pint_report* rep) {
  std::memset(reinterpret_cast<char*>(rep) + sizeof(size_t), 0, sizeof(pint_report) - sizeof(size_t));
  rep->status = status;
  rep->iterations = c.iter;
  rep->alpha_used = pl->alpha;
  rep->c_bar = c.c_bar;
  rep->est_rel_err = c.est;
  for (int k = 0; k < PINT_HIST && k < c.iter; ++k) {
    rep->upd_hist[k] = c.upd_hist[k];
    rep->res_hist[k] = c.res_hist[k];
  }
  rep->mass_drift = std::nan("");
  rep->energy_monotone = -1;
  rep->inner_iterations = 0;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* pint_status_string(int s) {
  switch (s) {
    case PINT_OK: return "PINT_OK";
    case PINT_EINVAL: return "PINT_EINVAL: invalid argument";
    case PINT_ENOCONV: return "PINT_ENOCONV: not converged within max_iter";
    case PINT_EDIVERGED: return "PINT_EDIVERGED: iteration diverged";
    case PINT_ENOMEM: return "PINT_ENOMEM: workspace or pool too small";
    case PINT_EHIP: return "PINT_EHIP: HIP runtime error";
    case PINT_ETIMEDOUT: return "PINT_ETIMEDOUT: timed out";
    case PINT_ECANCELED: return "PINT_ECANCELED: cancelled";
    case PINT_ENOTFOUND: return "PINT_ENOTFOUND: unknown ticket";
    default: return "unknown status";
  }
}

const char* pint_last_error(void) { return g_last_error.c_str(); }
const char* pint_version(void) { return "pint-mi355x 0.1 (gfx950)"; }

int pint_plan_create(const pint_problem* p, pint_plan** out) { return pint::plan_create_ex(p, pint::PlanOpts{}, out); }

}  // extern "C"

namespace pint {

int plan_create_ex(const pint_problem* p, const PlanOpts& opts, pint_plan** out) {
  if (!out) return set_err(nullptr, PINT_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p, nullptr);
  if (rc) return rc;
  pint_plan* pl = new (std::nothrow) pint_plan();
  if (!pl) return set_err(nullptr, PINT_ENOMEM, "host allocation failed");
  pl->p = *p;
  pl->p.struct_size = sizeof(pint_problem);
  pl->dim = p->dim;
  pl->n = p->nx;
  pl->nt = p->nt;
  pl->ns = p->dim == 2 ? p->nx * p->nx : p->nx;
  const double lx = p->lx > 0 ? p->lx : 1.0;
  pl->h = lx / p->nx;
  pl->dof = double(pl->ns) * pl->nt;
  pl->rtol = p->rtol > 0 ? p->rtol : 1e-10;
  pl->max_iter = p->max_iter > 0 ? p->max_iter : 30;
  pl->fp64 = p->precision == PINT_PREC_FP64;
  // BF16 keeps the FP64 forward spatial transform of the mixed mode
  pl->mixed = p->precision == PINT_PREC_MIXED || p->precision == PINT_PREC_BF16_REFINE;
  pl->dense = dense_kind_of(p);
  pl->norefine = p->precision == PINT_PREC_FP32_NOREFINE || p->precision == PINT_PREC_BF16_NOREFINE;
  pl->direct = p->dts != nullptr;
  {
    // tuning override of the time-solve tile width (spatial modes per workgroup)
    const char* tile = std::getenv("PINT_TIME_TILE");
    pl->time_tile = tile ? std::atoi(tile) : 0;
  }
  if (pl->direct) {
    pl->dts.assign(p->dts, p->dts + p->nt);
    pl->p.dts = nullptr;  // the caller's array is not kept
  }
  // Panels as wide as the forward column pass's row pieces (a 128-byte line;
  // 64 bytes for the mixed plan's FP64-to-FP32 pass) when the time-solve tile
  // is narrower (large N_t): the tile's levels then sit in one contiguous
  // range instead of N_t pieces spread over the whole array.  Measured per
  // iteration at 512^2 x 1024: FP32 3.89 -> 3.73 ms, FP64 6.09 -> 5.84 ms,
  // mixed 4.40 -> 4.29 ms; one-tile panels speed the time solve further but
  // slow the column passes' scattered pieces more (FP32 4.13 ms).
  pl->tps_spec = ilog2(pl->ns);
  if (pl->dim == 2 && pl->dense < 0 && !pl->direct) {
    const int m = time_tile_modes(pl->fp64, pl->nt, pl->ns, pl->time_tile);
    const int line = (pl->fp64 || pl->mixed) ? 16 : 32;
    if (m > 0 && m < line && line < pl->ns) {
      pl->tiled = true;
      pl->tps_spec = ilog2(line);
    }
  }
  pl->nbl = rows_blocks_per_level(pl->dim, pl->n);
  pl->nbl_f = rows_fwd_blocks_per_level(pl->dim, pl->n);
  if (pl->nt % rows_levels_per_block(pl->dim, pl->n) != 0) {
    delete pl;
    return set_err(nullptr, PINT_EINVAL, "nt must be a multiple of the 1D levels per block");
  }
  if (p->op == PINT_OP_CH || p->op == PINT_OP_CH_EYRE) pl->p.theta = 1.0;

  // Admissibility of alpha: the slowest-decaying (or fastest-growing) mode
  // multiplies the WR error by alpha R^{N_t} / (1 - alpha R^{N_t}) per sweep
  // (fully discrete analysis of Section 2.2, thm3; thm6 for the spinodal
  // case), R = R_theta(dt mu_min).  Require alpha R^{N_t} < 1/2.
  const double mmin = mu_min(pl->p, pl->dim, pl->n, pl->h);
  const double dt_max = pl->direct ? *std::max_element(pl->dts.begin(), pl->dts.end()) : p->dt;
  const double z = dt_max * mmin;
  const double th = pl->p.theta;
  const double R = (1.0 - (1.0 - th) * z) / (1.0 + th * z);
  if (!(1.0 + th * z > 0.0)) {
    delete pl;
    return set_err(nullptr, PINT_EINVAL, "1 + theta dt mu_min <= 0: the sequential scheme is singular");
  }
  const double RN = std::pow(std::fabs(R) > 1.0 ? std::fabs(R) : 1.0, pl->nt);
  if (pl->direct) {
    pl->alpha = 0.0;  // no alpha-circulant preconditioner: the pencil is diagonalized directly
  } else if (p->alpha == 0.0) {
    double al = 1e-3;
    if (al * RN > 0.1) al = 0.1 / RN;
    pl->alpha = al;
  } else {
    if (p->alpha * RN >= 0.5) {
      delete pl;
      return set_err(nullptr, PINT_EINVAL,
                     "alpha * R^Nt >= 1/2: alpha is not admissible for this problem (choose alpha = 0 for auto)");
    }
    pl->alpha = p->alpha;
  }
  pl->p.alpha = pl->alpha;
  pl->a = pl->direct ? 1.0 : std::exp(std::log(pl->alpha) / pl->nt);

  // residual coefficients
  ResidArgs& ra = pl->ra;
  ra.inv_dt = 1.0 / p->dt;
  ra.inv_h2 = 1.0 / (pl->h * pl->h);
  ra.theta = pl->p.theta;
  const double e2 = p->eps * p->eps;
  switch (p->op) {
    case PINT_OP_BIHARMONIC: ra.c3 = 0; ra.c1 = 0; ra.c1p = 0; ra.c2 = -1.0; break;
    case PINT_OP_LINEAR_CH: ra.c3 = 0; ra.c1 = -p->beta * p->beta; ra.c1p = 0; ra.c2 = -e2; break;
    case PINT_OP_CH: ra.c3 = 1; ra.c1 = -1.0; ra.c1p = 0; ra.c2 = -e2; break;
    default: ra.c3 = 1; ra.c1 = 0; ra.c1p = -1.0; ra.c2 = -e2; break;
  }

  HostTables t;
  build_tables(pl, t);
  std::vector<unsigned char>& buf = pl->host_tab;
  store_offs(put_all<double>(buf, t), pl->offs_d);
  store_offs(put_all<float>(buf, t), pl->offs_f);
  reserve_dense(buf, pl->dense >= 0 ? pl->dense : (pl->direct ? DK_F32 : -1), pl->nt, pl->offs_w);
  if (pl->dense >= 0 && !pl->direct) put_dense(buf, pl, pl->offs_w);
  if (pl->direct) reserve_direct(buf, pl);
  pl->tab_bytes = align256(buf.size());
  if (!opts.defer_tables) {
    void* mem = opts.d_tables;
    if (!mem) {
      hipError_t e = hipMalloc(&mem, pl->tab_bytes);
      if (e != hipSuccess) {
        rc = hip_fail(nullptr, e, "hipMalloc(tables)");
        delete pl;
        return rc;
      }
      pl->d_tab = mem;  // owned
      e = hipMemcpy(mem, buf.data(), buf.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        rc = hip_fail(nullptr, e, "table copy");
        delete pl;
        return rc;
      }
      rc = plan_bind_tables(pl, mem, nullptr, false);
      if (!rc && pl->direct) {
        // the eigendecomposition ran on the null stream: finish it here
        e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = hip_fail(nullptr, e, "time-step eigendecomposition");
      }
      if (rc) {
        delete pl;
        return rc;
      }
    } else {
      rc = plan_bind_tables(pl, mem, opts.stream, true);
      if (rc) {
        delete pl;
        return rc;
      }
    }
  }
  if (opts.host_mirror) {
    const hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&pl->h_ctrl), sizeof(Ctrl), hipHostMallocCoherent);
    if (e != hipSuccess) {
      rc = hip_fail(nullptr, e, "hipHostMalloc(status mirror)");
      delete pl;
      return rc;
    }
  }
  *out = pl;
  return PINT_OK;
}

int plan_bind_tables(pint_plan* pl, void* d_mem, hipStream_t st, bool copy) {
  if (pl->d_tab && pl->own_tab && pl->d_tab != d_mem) (void)hipFree(pl->d_tab);
  pl->d_tab = d_mem;
  pl->own_tab = !copy;  // a copied-into block belongs to the caller
  if (copy) {
    hipError_t e = hipMemcpyAsync(d_mem, pl->host_tab.data(), pl->host_tab.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(pl, e, "table copy");
  }
  unsigned char* base = static_cast<unsigned char*>(d_mem);
  bind<double>(load_offs(pl->offs_d), base, pl, pl->dtd, pl->tad);
  bind<float>(load_offs(pl->offs_f), base, pl, pl->dtf, pl->taf);
  pl->dargs = DenseArgs{};
  pl->ra.inv_dts = nullptr;
  if (pl->direct) {
    // the FP64 eigendecomposition of the time-step pencil, on the GPU
    pl->dargs.direct = 1;
    pl->dargs.wf = reinterpret_cast<const float*>(base + pl->offs_w[0]);
    pl->dargs.wb = reinterpret_cast<const float*>(base + pl->offs_w[1]);
    pl->dargs.w64 = reinterpret_cast<const double*>(base + pl->off_w64);
    pl->dargs.v64 = reinterpret_cast<const double*>(base + pl->off_v64);
    pl->ra.inv_dts = reinterpret_cast<const double*>(base + pl->off_idts);
    EigArgs ea{reinterpret_cast<const double*>(base + pl->off_dts), pl->p.theta, pl->nt,
               reinterpret_cast<double*>(base + pl->off_v64), reinterpret_cast<double*>(base + pl->off_w64),
               reinterpret_cast<cx<double>*>(base + pl->offs_d[4]), reinterpret_cast<cx<float>*>(base + pl->offs_f[4]),
               reinterpret_cast<float*>(base + pl->offs_w[0]), reinterpret_cast<float*>(base + pl->offs_w[1])};
    const hipError_t e = launch_eig_steps(ea, st);
    if (e != hipSuccess) return hip_fail(pl, e, "time-step eigendecomposition kernel");
  } else if (pl->dense == DK_F32) {
    pl->dargs.wf = reinterpret_cast<const float*>(base + pl->offs_w[0]);
    pl->dargs.wb = reinterpret_cast<const float*>(base + pl->offs_w[1]);
  } else if (pl->dense >= 0) {
    pl->dargs.wf_hi = base + pl->offs_w[0];
    pl->dargs.wf_lo = base + pl->offs_w[1];
    pl->dargs.wb_hi = base + pl->offs_w[2];
    pl->dargs.wb_lo = base + pl->offs_w[3];
  }
  return PINT_OK;
}

size_t plan_table_bytes(const pint_problem* p) {
  // the table block depends only on N, N_t and the time path
  HostTables t;
  t.tw_s.resize(p->nx);
  t.wq.resize(p->nx);
  t.wi.resize(p->nx);
  t.tw_t.resize(p->nt);
  t.lam1.resize(p->nt);
  t.pco.resize(p->nt);
  t.qco.resize(p->nt);
  t.aj.resize(p->nt);
  t.aij.resize(p->nt);
  t.lamx.resize(p->nx);
  t.lamy.resize(p->dim == 2 ? p->nx : 1);
  std::vector<unsigned char> buf;
  put_all<double>(buf, t);
  put_all<float>(buf, t);
  size_t offs[4];
  reserve_dense(buf, dense_kind_of(p) >= 0 ? dense_kind_of(p) : (p->dts ? DK_F32 : -1), p->nt, offs);
  if (p->dts) {
    // the layout of reserve_direct
    std::vector<double> steps(p->nt);
    put_re<double>(buf, buf.size(), steps);
    put_re<double>(buf, buf.size(), steps);
    buf.resize(align256(buf.size()) + size_t(p->nt) * p->nt * 8);
    buf.resize(align256(buf.size()) + size_t(p->nt) * p->nt * 8);
  }
  return align256(buf.size());
}

size_t plan_workspace_bytes(const pint_plan* pl) { return work_size(pl); }
int plan_max_iter(const pint_plan* pl) { return pl->max_iter; }
int plan_nt(const pint_plan* pl) { return pl->nt; }
int plan_ns(const pint_plan* pl) { return pl->ns; }

int solve_begin(pint_plan* pl, const double* d_u0, double* d_U, void* d_work, size_t work_bytes, hipStream_t st,
                Ctrl* host) {
  Work w;
  int rc = carve(pl, d_work, work_bytes, w);
  if (rc) return rc;
  return begin_solve(pl, d_u0, d_U, w, st, host);
}

int solve_enqueue(pint_plan* pl, const double* d_u0, double* d_U, void* d_work, size_t work_bytes, hipStream_t st,
                  Ctrl* host, int it) {
  Work w;
  int rc = carve(pl, d_work, work_bytes, w);
  if (rc) return rc;
  const bool bcast = (pl->p.flags & PINT_FLAG_INIT_BROADCAST_U0) != 0;
  return enqueue_any(pl, d_u0, d_U, w, st, nullptr, bcast && it == 0, host);
}

int solve_status(const pint_plan* pl, const Ctrl& c, pint_report* rep) {
  const int status = c.done ? c.status : PINT_ENOCONV;
  if (rep) fill_report(pl, c, status, rep);
  return status;
}

}  // namespace pint

extern "C" {



int pint_plan_destroy(pint_plan* plan) {
  delete plan;
  return PINT_OK;
}

const char* pint_plan_last_error(const pint_plan* plan) { return plan ? plan->err.c_str() : ""; }

int pint_plan_workspace_size(const pint_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return set_err(nullptr, PINT_EINVAL, "NULL argument");
  *bytes = work_size(plan);
  return PINT_OK;
}

int pint_plan_alpha(const pint_plan* plan, double* alpha) {
  if (!plan || !alpha) return set_err(nullptr, PINT_EINVAL, "NULL argument");
  *alpha = plan->alpha;
  return PINT_OK;
}

int pint_solve(pint_plan* pl, const double* d_u0, double* d_U, void* d_work, size_t work_bytes, void* stream,
               pint_report* rep) {
  if (!pl) return set_err(nullptr, PINT_EINVAL, "plan is NULL");
  if (!d_u0 || !d_U) return set_err(&pl->err, PINT_EINVAL, "u0/U pointer is NULL");
  if (rep && rep->struct_size < sizeof(pint_report))
    return set_err(&pl->err, PINT_EINVAL, "pint_report.struct_size too small");
  auto t0 = std::chrono::steady_clock::now();
  Work w;
  int rc = carve(pl, d_work, work_bytes, w);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool timing = (pl->p.flags & PINT_FLAG_STAGE_TIMING) != 0;
  if (timing && pl->ev.size() < size_t(EV_PER_IT * pl->max_iter)) {
    while (pl->ev.size() < size_t(EV_PER_IT * pl->max_iter)) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e), "hipEventCreate");
      pl->ev.push_back(e);
    }
  }
  if (field_mode(pl)) {
    int inner = 0;
    rc = solve_field(pl, d_u0, d_U, d_work, work_bytes, w, st, &inner);
    if (rc) return rc;
    const Ctrl& c = *pl->h_ctrl;
    const int status = c.done ? c.status : PINT_ENOCONV;
    if (rep) {
      fill_report(pl, c, status, rep);
      rep->inner_iterations = inner;
      rep->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status != PINT_OK)
      set_err(&pl->err, status, status == PINT_ENOCONV ? "not converged within max_iter" : "iteration diverged");
    return status;
  }
  const bool bcast = (pl->p.flags & PINT_FLAG_INIT_BROADCAST_U0) != 0;
  // Enqueue as many iterations as the previous solve of this plan needed
  // (kernels after the device stop flag is set return at once), then check
  // the flag after each further iteration.
  int it = 0;
  const int first_check = std::min(std::max(pl->predict, 2), pl->max_iter);
  const bool use_graph = (pl->p.flags & PINT_FLAG_SOLVE_GRAPH) && !timing && st != nullptr;
  if (use_graph) {
    // init + the predicted iterations as one graph, captured once per
    // (buffers, stream, iteration count) and replayed afterwards
    if (!(pl->gexec && pl->g_u0 == d_u0 && pl->g_U == d_U && pl->g_work == d_work && pl->g_st == st &&
          pl->g_iters == first_check)) {
      if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
      pl->gexec = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      int rc2 = begin_solve(pl, d_u0, d_U, w, st, pl->h_ctrl);
      for (int k = 0; k < first_check && !rc2; ++k)
        rc2 = enqueue_any(pl, d_u0, d_U, w, st, nullptr, bcast && k == 0, pl->h_ctrl);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(st, &g);
      if (rc2) {
        if (g) (void)hipGraphDestroy(g);
        return rc2;
      }
      if (e != hipSuccess) return hip_fail(pl, e, "hipStreamEndCapture");
      const hipError_t e2 = hipGraphInstantiate(&pl->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e2 != hipSuccess) {
        pl->gexec = nullptr;
        return hip_fail(pl, e2, "hipGraphInstantiate");
      }
      pl->g_u0 = d_u0;
      pl->g_U = d_U;
      pl->g_work = d_work;
      pl->g_st = st;
      pl->g_iters = first_check;
    }
    HIPCHK(hipGraphLaunch(pl->gexec, st), "hipGraphLaunch");
    it = first_check;
    HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (reinterpret_cast<volatile int&>(pl->h_ctrl->done)) it = pl->max_iter + 1;  // finished inside the graph
  } else {
    rc = begin_solve(pl, d_u0, d_U, w, st, pl->h_ctrl);
    if (rc) return rc;
  }
  for (; it < pl->max_iter; ++it) {
    hipEvent_t* evs = timing ? &pl->ev[EV_PER_IT * it] : nullptr;
    rc = enqueue_any(pl, d_u0, d_U, w, st, evs, bcast && it == 0, pl->h_ctrl);
    if (rc) return rc;
    if (it + 1 >= first_check) {
      HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
      if (reinterpret_cast<volatile int&>(pl->h_ctrl->done)) {
        ++it;
        break;
      }
    }
  }
  const bool invariants = (pl->p.flags & PINT_FLAG_INVARIANTS) != 0;
  if (invariants) {
    // mass and energy of u_0..u_{N_t}; the block partials are free scratch now
    DiagArgs da{d_U, nullptr, nullptr, pl->n, pl->ns, pl->dim, pl->p.eps * pl->p.eps, 1.0 / (pl->h * pl->h),
                pl->dim == 2 ? pl->h * pl->h : pl->h};
    const bool ch = pl->p.op == PINT_OP_CH || pl->p.op == PINT_OP_CH_EYRE;
    HIPCHK(launch_invariants(da, d_u0, w.part, pl->nt, ch, w.ctrl, pl->h_ctrl, st), "invariants kernels");
  }
  HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
  const Ctrl& c = *pl->h_ctrl;
  const int status = c.done ? c.status : PINT_ENOCONV;
  if (status == PINT_OK) pl->predict = c.iter;
  if (rep) {
    fill_report(pl, c, status, rep);
    if (invariants) {
      rep->mass_drift = c.mass_drift;
      rep->energy_monotone = c.energy_ok;
    }
    if (timing) {
      for (int k = 0; k < c.iter && k < it; ++k)
        for (int s = 0; s < EV_PER_IT / 2; ++s) {
          float ms = 0.f;  // stages without a kernel (the column passes in 1D) stay 0
          if (hipEventElapsedTime(&ms, pl->ev[EV_PER_IT * k + 2 * s], pl->ev[EV_PER_IT * k + 2 * s + 1]) ==
              hipSuccess)
            rep->ms_stage[s] += ms;
        }
    }
    rep->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status != PINT_OK) {
    set_err(&pl->err, status, status == PINT_ENOCONV ? "not converged within max_iter" : "iteration diverged");
  }
  return status;
}

}  // extern "C"

// ------------------------------------------------------------ no-alloc solve
// A file-scope device array serves as the workspace of pint_solve_noalloc.
// Each device that loads the library holds its own copy until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host it
// names a stand-in, not device memory): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[PINT_NOALLOC_WORKSPACE_BYTES];

namespace {
constexpr size_t kNoallocBytes = size_t(PINT_NOALLOC_WORKSPACE_BYTES);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_err(nullptr, PINT_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_err(nullptr, PINT_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_err(nullptr, PINT_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PINT_OK;
}
}  // namespace

extern "C" {

int pint_solve_noalloc(pint_plan* pl, const double* d_u0, double* d_U, void* stream, pint_report* rep) {
  if (!pl) return set_err(nullptr, PINT_EINVAL, "plan is NULL");
  if (pl->p.flags & (PINT_FLAG_SOLVE_GRAPH | PINT_FLAG_STAGE_TIMING))
    return set_err(&pl->err, PINT_EINVAL,
                   "pint_solve_noalloc takes no PINT_FLAG_SOLVE_GRAPH or PINT_FLAG_STAGE_TIMING (both create "
                   "runtime objects)");
  const size_t need = work_size(pl);
  if (need > kNoallocBytes)
    return set_err(&pl->err, PINT_ENOMEM,
                   "problem needs " + std::to_string(need) + " bytes of workspace; the static workspace of "
                   "pint_solve_noalloc holds " + std::to_string(kNoallocBytes));
  void* work = nullptr;
  const int rc = scratch_for_current_device(&work);
  if (rc) {
    pl->err = g_last_error;
    return rc;
  }
  return pint_solve(pl, d_u0, d_U, work, kNoallocBytes, stream, rep);
}

int pint_residual(pint_plan* pl, const double* d_u0, const double* d_U, double* d_r, void* d_work,
                  size_t work_bytes, void* stream) {
  if (!pl || !d_u0 || !d_U || !d_r) return set_err(pl ? &pl->err : nullptr, PINT_EINVAL, "NULL argument");
  Work w;
  int rc = carve(pl, d_work, work_bytes, w);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  ResidArgs ra = pl->ra;
  ra.u0 = d_u0;
  ra.U = d_U;
  ra.part = w.part;
  ra.done = nullptr;
  ra.bcast = 0;
  HIPCHK((launch_rows_fwd<double, double>(pl->dim, pl->n, ra, nullptr, d_r, pl->dtd, pl->nt, 1, st)),
         "residual kernel");
  return PINT_OK;
}

int pint_dct(pint_plan* pl, const void* d_in, void* d_out, int inverse, void* stream) {
  if (!pl || !d_in || !d_out) return set_err(pl ? &pl->err : nullptr, PINT_EINVAL, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(d_in) | reinterpret_cast<uintptr_t>(d_out)) & 15)
    return set_err(&pl->err, PINT_EINVAL, "DCT buffers must be 16-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (pl->fp64)
    HIPCHK(launch_dct<double>(pl->dim, pl->n, static_cast<const double*>(d_in), static_cast<double*>(d_out), pl->dtd,
                              pl->nt, inverse != 0, st),
           "dct kernel");
  else
    HIPCHK(launch_dct<float>(pl->dim, pl->n, static_cast<const float*>(d_in), static_cast<float*>(d_out), pl->dtf,
                             pl->nt, inverse != 0, st),
           "dct kernel");
  return PINT_OK;
}

int pint_time_solve(pint_plan* pl, void* d_S, double c_bar, void* stream) {
  if (!pl || !d_S) return set_err(pl ? &pl->err : nullptr, PINT_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_S) & 15)
    return set_err(&pl->err, PINT_EINVAL, "time-solve buffer must be 16-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (pl->fp64) {
    TimeArgs<double> ta = pl->tad;
    ta.cbar_val = c_bar;
    e = launch_time_any<double>(pl, static_cast<double*>(d_S), ta, st);
  } else {
    TimeArgs<float> ta = pl->taf;
    ta.cbar_val = c_bar;
    e = launch_time_any<float>(pl, static_cast<float*>(d_S), ta, st);
  }
  if (e != hipSuccess) return hip_fail(pl, e, "time-solve kernel");
  return PINT_OK;
}

int pint_precond_apply(pint_plan* pl, const double* d_r, double* d_delta, double c_bar, void* d_work,
                       size_t work_bytes, void* stream) {
  if (!pl || !d_r || !d_delta) return set_err(pl ? &pl->err : nullptr, PINT_EINVAL, "NULL argument");
  Work w;
  int rc = carve(pl, d_work, work_bytes, w);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)pl->nt * pl->ns;
  UpdArgs ua{nullptr, nullptr, w.part, nullptr, 0};
  if (pl->fp64) {
    double* S = static_cast<double*>(w.S);
    HIPCHK((launch_cast<double, double>(d_r, S, n, st)), "cast");
    HIPCHK(launch_dct<double>(pl->dim, pl->n, S, S, pl->dtd, pl->nt, false, st), "dct");
  } else if (pl->mixed) {
    // FP64 forward transform, rounded to FP32 after the last forward pass
    double* S64 = static_cast<double*>(w.S64);
    float* S = static_cast<float*>(w.S);
    HIPCHK((launch_cast<double, double>(d_r, S64, n, st)), "cast");
    if (pl->dim == 2) {
      HIPCHK(launch_dct<double>(1, pl->n, S64, S64, pl->dtd, pl->nt * pl->n, false, st), "x-dct");
      HIPCHK((launch_cols<double, float>(pl->n, S64, S, nullptr, pl->dtd, pl->nt, false, st, ilog2(pl->ns),
                                         ilog2(pl->ns))),
             "y-dct");
    } else {
      HIPCHK(launch_dct<double>(1, pl->n, S64, S64, pl->dtd, pl->nt, false, st), "x-dct");
      HIPCHK((launch_cast<double, float>(S64, S, n, st)), "cast");
    }
  } else {
    float* S = static_cast<float*>(w.S);
    HIPCHK((launch_cast<double, float>(d_r, S, n, st)), "cast");
    HIPCHK(launch_dct<float>(pl->dim, pl->n, S, S, pl->dtf, pl->nt, false, st), "dct");
  }
  rc = pint_time_solve(pl, w.S, c_bar, stream);
  if (rc) return rc;
  if (pl->fp64) {
    double* S = static_cast<double*>(w.S);
    if (pl->dim == 2)
      HIPCHK((launch_cols<double, double>(pl->n, S, S, nullptr, pl->dtd, pl->nt, true, st, ilog2(pl->ns),
                                          ilog2(pl->ns))),
             "inverse y-dct");
    HIPCHK(launch_rows_inv<double>(pl->dim, pl->n, ua, S, d_delta, pl->dtd, pl->nt, 1, st), "inverse x-dct");
  } else {
    float* S = static_cast<float*>(w.S);
    if (pl->dim == 2)
      HIPCHK((launch_cols<float, float>(pl->n, S, S, nullptr, pl->dtf, pl->nt, true, st, ilog2(pl->ns),
                                        ilog2(pl->ns))),
             "inverse y-dct");
    HIPCHK(launch_rows_inv<float>(pl->dim, pl->n, ua, S, d_delta, pl->dtf, pl->nt, 1, st), "inverse x-dct");
  }
  return PINT_OK;
}

int pint_field_jacobian_solve(pint_plan* pl, const double* d_u0, const double* d_U, const double* d_r,
                              double* d_delta, double inner_rtol, int inner_max, void* d_work, size_t work_bytes,
                              void* stream, int* inner_iterations) {
  if (!pl || !d_u0 || !d_U || !d_r || !d_delta) return set_err(pl ? &pl->err : nullptr, PINT_EINVAL, "NULL argument");
  if (!field_mode(pl)) return set_err(&pl->err, PINT_EINVAL, "the plan lacks PINT_FLAG_FIELD_JACOBIAN");
  if (!(inner_rtol > 0.0) || inner_max < 1) return set_err(&pl->err, PINT_EINVAL, "inner_rtol > 0, inner_max >= 1");
  Work w;
  int rc = carve(pl, d_work, work_bytes, w);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  FieldWork f;
  field_carve(pl, d_work, f);
  const size_t n = size_t(pl->nt) * pl->ns;
  HIPCHK(launch_jfield(d_U, f.jfield, pl->nt, pl->ns, st), "field kernel");
  std::vector<double> j(pl->ns);
  HIPCHK(hipMemcpyAsync(j.data(), f.jfield, j.size() * sizeof(double), hipMemcpyDeviceToHost, st), "field copy");
  HIPCHK(hipMemcpyAsync(f.v[0], d_r, n * sizeof(double), hipMemcpyDeviceToDevice, st), "residual copy");
  HIPCHK(hipStreamSynchronize(st), "hipStreamSynchronize");
  double cbar = 0.0;
  for (double x : j) cbar += x;
  cbar /= double(pl->ns);
  PinnedDots hd;
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hd.p), 4 * DOT_BLOCKS * sizeof(double), hipHostMallocDefault),
         "hipHostMalloc(dot partials)");
  int iters = 0;
  rc = field_inner_solve(pl, d_u0, f, f.v[0], d_delta, cbar, inner_rtol, inner_max, d_work, work_bytes, st, hd.p,
                         &iters);
  if (inner_iterations) *inner_iterations = iters;
  return rc;
}

int pint_time_eig(pint_plan* pl, double* h_V, double* h_W, double* h_d) {
  if (!pl || !h_V || !h_W || !h_d) return set_err(pl ? &pl->err : nullptr, PINT_EINVAL, "NULL argument");
  if (!pl->direct) return set_err(&pl->err, PINT_EINVAL, "the plan has uniform steps (no direct diagonalization)");
  HIPCHK(hipDeviceSynchronize(), "hipDeviceSynchronize");
  const unsigned char* base = static_cast<const unsigned char*>(pl->d_tab);
  const size_t mat = size_t(pl->nt) * pl->nt * sizeof(double);
  HIPCHK(hipMemcpy(h_V, base + pl->off_v64, mat, hipMemcpyDeviceToHost), "copy V");
  HIPCHK(hipMemcpy(h_W, base + pl->off_w64, mat, hipMemcpyDeviceToHost), "copy W");
  std::vector<std::complex<double>> lam(pl->nt);
  HIPCHK(hipMemcpy(lam.data(), base + pl->offs_d[4], pl->nt * sizeof(std::complex<double>), hipMemcpyDeviceToHost),
         "copy d");
  for (int j = 0; j < pl->nt; ++j) h_d[j] = lam[j].real();
  return PINT_OK;
}

int pint_diagnostics(pint_plan* pl, const double* d_U, double* d_mass, double* d_energy, void* stream) {
  if (!pl || !d_U || !d_mass || !d_energy) return set_err(pl ? &pl->err : nullptr, PINT_EINVAL, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  DiagArgs a{d_U, d_mass, d_energy, pl->n, pl->ns, pl->dim, pl->p.eps * pl->p.eps, 1.0 / (pl->h * pl->h),
             pl->dim == 2 ? pl->h * pl->h : pl->h};
  HIPCHK(launch_diagnostics(a, pl->nt, st), "diagnostics kernel");
  return PINT_OK;
}

}  // extern "C"
