// Internal interface between the host runtime and the kernels: argument
// blocks, the device control record and the launcher declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stddef.h>

#include "device_common.hpp"

namespace pint {

// Stage timing: when set, the next kernel launch of this thread is bracketed by
// these events, stamped by the dispatch itself (hipExtLaunchKernelGGL), so the
// elapsed time is the kernel's own duration.  A launch consumes them.
extern thread_local hipEvent_t g_launch_ev0, g_launch_ev1;
inline void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_launch_ev0 = start;
  g_launch_ev1 = stop;
}
#define PINT_LAUNCH(K, G, B, S, ST, ...)                                                              \
  do {                                                                                                \
    if (::pint::g_launch_ev0) {                                                                       \
      hipEvent_t e0_ = ::pint::g_launch_ev0, e1_ = ::pint::g_launch_ev1;                               \
      ::pint::g_launch_ev0 = ::pint::g_launch_ev1 = nullptr;                                          \
      hipExtLaunchKernelGGL(K, G, B, S, ST, e0_, e1_, 0, __VA_ARGS__);                                \
    } else {                                                                                          \
      hipLaunchKernelGGL(K, G, B, S, ST, __VA_ARGS__);                                                \
    }                                                                                                 \
  } while (0)

constexpr int PINT_HIST_DEV = 64;
// status codes mirrored from the public header (kept in sync by a static_assert
// in the runtime)
constexpr int PINT_OK_DEV = 0;

// Per-level partial results written by the per-slice kernels.
enum : int {
  PART_RSQ = 0,   // sum r_n^2           (residual kernel)
  PART_DSQ = 1,   // sum delta_n^2       (update kernel)
  PART_USQ = 2,   // sum u_n^2 after the update
  PART_U2 = 3,    // sum 3 u_n^2 after the update (scalar Jacobian)
  PART_DMAX = 4,  // max |delta_n|
  PART_STRIDE = 8
};

// Device-resident control record of one solve.
struct Ctrl {
  int iter;      // completed outer iterations
  int done;      // nonzero: stop (converged, diverged or out of iterations)
  int status;    // PINT_OK / PINT_ENOCONV / PINT_EDIVERGED
  int pad;
  double c_bar;  // scalar averaged Jacobian for the next time solve
  double upd_prev, upd_first, est;
  double upd_hist[PINT_HIST_DEV];
  double res_hist[PINT_HIST_DEV];
  double mass_drift;  // invariants of the final iterate (k_invariants_fin)
  int energy_ok;      // 1 monotone, 0 violated, -1 not applicable
  int pad2;
};

struct ResidArgs {
  const double* u0;
  const double* U;
  double* part;     // [level][block] partials
  const int* done;
  const double* inv_dts;  // 1/dt_n per level (nonuniform steps), or null: inv_dt
  double inv_dt, inv_h2, theta;
  double c1, c1p, c2, c3;
  int bcast;        // the iterate is u0 at every level (first iteration)
  // Linearized operator (approximate Jacobian of eq. approx_jacobian): with
  // jfield non-null the cubic term c3 v^3 becomes jfield(x) v, and with wrap
  // the predecessor of level 1 is wrap_alpha u_{N_t} (the alpha-circulant
  // corner) instead of u0.
  const double* jfield;
  int wrap, nt;
  double wrap_alpha;
  // With bcast in 2D every level's residual is the same: the launch covers
  // level 0 only and its blocks write their partial sums for all nt levels.
  int one_level;
};

struct FinArgs {
  Ctrl* ctrl;
  Ctrl* host;  // pinned host mirror of the status fields (nullable)
  const double* part;
  double* fin;   // per-group reductions [finalize_groups][4] (two-stage finalize)
  int nt, nbl, max_iter;
  int nbl_f;     // blocks per level of the forward row pass (its residual partials)
  int stagnate;  // unrefined mode: also stop once the update stops contracting
  double dof, rtol, safety;
};

struct UpdArgs {
  double* U;
  const double* u0;
  double* part;
  const int* done;
  int bcast;        // U_n = u0 + delta_n instead of U_n += delta_n
  int round32;      // store U_n rounded to FP32 (unrefined mode)
};

template <typename T>
struct DctTables {
  const cx<T>* tw;  // exp(-2 pi i m / N), m < N
  const cx<T>* wq;  // s_k exp(-i pi k / (2N))
  const cx<T>* wi;  // exp(+i pi k / (2N)) / s_k
};

template <typename T>
struct TimeArgs {
  const cx<T>* tw;    // exp(-2 pi i m / N_t)
  const cx<T>* lam1;  // (1 - a w^l) / dt
  const cx<T>* pco;   // coefficient of lam_k in sigma (before - c_bar)
  const cx<T>* qco;   // coefficient of lam_k^2 in sigma
  const T* aj;        // a^j
  const T* aij;       // a^{-j} / N_t
  const T* lamx;      // 1D Laplacian spectrum along x
  const T* lamy;      // along y (1D: a single 0)
  const double* cbar; // device scalar (used when non-null)
  double cbar_val;    // value used when cbar is null
  const int* done;
  int nx, ns, cbar_mode;
  int tile;           // cap on the spatial modes per workgroup (0 = automatic)
  int tps;            // log2 of the spectral panel width P: mode k of level n
                      // at ((k / P) N_t + n) P + k mod P (P = ns: [level][mode])
  int bcast_in;       // every level's input is level 0's (read level 0 only)
};

struct InitArgs {
  const double* u0;
  const double* U;
  double* part;
  int nt, ns, nbl, broadcast;
};

struct DiagArgs {
  const double* U;
  double* mass;
  double* energy;
  int nx, ns, dim;
  double eps2, inv_h2, hd;
};

// Row blocks per level of the 2D row passes (1 in 1D), and levels per block
// of the 1D row passes (1 in 2D).
int rows_blocks_per_level(int dim, int n);
// Blocks per level of the forward (residual) row pass, which may use narrower
// blocks than the inverse pass.
int rows_fwd_blocks_per_level(int dim, int n);
int rows_levels_per_block(int dim, int n);

// Forward row pass: residual in RT arithmetic (double; float for the
// unrefined mode), x-DCT computed in T, stored in TO.
template <typename T, typename TO, typename RT = double>
hipError_t launch_rows_fwd(int dim, int n, const ResidArgs& a, TO* S, double* rout, const DctTables<T>& dt, int nt,
                           int mode, hipStream_t st);
template <typename T>
hipError_t launch_rows_inv(int dim, int n, const UpdArgs& a, const T* S, double* dout, const DctTables<T>& dt,
                           int nt, int mode, hipStream_t st);
// Column pass computing in T, reading Sin (T) and writing Sout (TO; TO == T
// for the inverse).  tps_in / tps_out: log2 of the panel width of each side's
// layout (log2(n^2): plain [level][mode]).  Sin == Sout is allowed when
// TO == T and the two layouts are the same.
template <typename T, typename TO>
hipError_t launch_cols(int n, const T* Sin, TO* Sout, const int* done, const DctTables<T>& dt, int nt, bool inv,
                       hipStream_t st, int tps_in, int tps_out, int levels = -1);
// Spatial modes per workgroup of the FFT time solve (its panel width when
// the spectral array is tiled).
int time_tile_modes(bool fp64, int nt, int ns, int tile);
template <typename T>
hipError_t launch_dct(int dim, int n, const T* in, T* out, const DctTables<T>& dt, int nt, bool inv,
                      hipStream_t st);
template <typename T>
hipError_t launch_time(int nt, T* S, const TimeArgs<T>& ta, hipStream_t st);

// Dense time contraction on the matrix cores (FP32 S, in place).  The W tables
// are N_t x N_t: for DK_F32 transposed FP32 copies ([k][m]) of W_f and W_b, for
// the BF16 kinds row-major BF16 hi / lo parts.
enum DenseKind { DK_F32 = 0, DK_BF16 = 1, DK_BF16X3 = 2 };
struct DenseArgs {
  const float* wf;   // W_f^T (DK_F32)
  const float* wb;   // W_b^T (DK_F32)
  const void* wf_hi; // BF16 W_f, hi / lo parts (BF16 kinds)
  const void* wf_lo;
  const void* wb_hi;
  const void* wb_lo;
  // direct diagonalization (nonuniform steps): rows of W_f y are eigen-
  // coordinates, each divided by the real lam1[j] + (pco[j] - c_bar) lam_k +
  // qco[j] lam_k^2 instead of the complex pair divide
  int direct;
  const double* w64;  // FP64 W_f [j][n] (rows: left eigenvectors; FP64 path)
  const double* v64;  // FP64 W_b [n][j] (columns: right eigenvectors)
};
// FP64 eigendecomposition of the theta-method time-step pencil with steps
// dts (B = diag(1/dt)(I - S), C = theta I + (1-theta) S): eigenvalues
// d_j = 1/(theta dt_j), unit-norm right eigenvectors V[:, j] and left ones
// W[j, :] with W C V = I; also the FP32 transposed copies used by the
// matrix-core contraction and the divide's eigenvalue tables.
struct EigArgs {
  const double* dts;
  double theta;
  int nt;
  double* v64;        // [n][j]
  double* w64;        // [j][n]
  cx<double>* lam1d;  // d_j (real part)
  cx<float>* lam1f;
  float* wfT;         // [n][j] = W[j][n]
  float* wbT;         // [j][n] = V[n][j]
};
hipError_t launch_eig_steps(const EigArgs& a, hipStream_t st);
// Direct-diagonalization time solve in FP64 (vector FMA), in place on S.
hipError_t launch_time_direct64(int nt, double* S, const TimeArgs<double>& ta, const DenseArgs& da,
                                hipStream_t st);
// Spatial modes per workgroup of the dense path (0 if N_t is too small).
int dense_cols_per_block(int nt);
hipError_t launch_time_dense(int kind, int nt, float* S, const TimeArgs<float>& ta, const DenseArgs& da,
                             hipStream_t st);
template <typename TI, typename TO>
hipError_t launch_cast(const TI* in, TO* out, size_t n, hipStream_t st);
hipError_t launch_finalize(const FinArgs& f, hipStream_t st);
// Workgroups of the first stage of the control reduction (0: one stage).
int finalize_groups(int nt, int nbl, int nbl_f);
// Reset the control record (and its host mirror); with need_cbar, also the
// first iteration's scalar averaged Jacobian.  The partials of the c_bar
// reduction use a.part (nparts <= ceil(total / 4096) slots).
hipError_t launch_init(const InitArgs& a, Ctrl* c, Ctrl* host, double dof, bool need_cbar, hipStream_t st);
hipError_t launch_diagnostics(const DiagArgs& a, int nt, hipStream_t st);
// Space-varying averaged Jacobian field j(x) = (1/N_t) sum_n 3 u_n(x)^2.
hipError_t launch_jfield(const double* U, double* j, int nt, int ns, hipStream_t st);
// out = a x + b y + c z (z may be null), n values.
hipError_t launch_axpbypcz(double* out, double a, const double* x, double b, const double* y, double c,
                           const double* z, size_t n, hipStream_t st);
// Partial sums of x_i y_i for `pairs` pairs in fixed-order blocks:
// partial[q * DOT_BLOCKS + block].
constexpr int DOT_BLOCKS = 512;
hipError_t launch_dots(const double* const* xs, const double* const* ys, int pairs, size_t n, double* partial,
                       hipStream_t st);
// U = (bcast ? u0 : U) + delta level by level, with the update partials of
// [level][block] (block = a 1/nbl share of the level) for the control kernel.
hipError_t launch_update_plain(double* U, const double* u0, const double* delta, double* part, int nt, int ns,
                               int nbl, int bcast, hipStream_t st);
// Mass drift and energy monotonicity of u_0, u_1..u_{N_t} into the control
// record and its host mirror; `scratch` holds 3 (N_t + 1) doubles.
hipError_t launch_invariants(const DiagArgs& a, const double* u0, double* scratch, int nt, bool energy, Ctrl* c,
                             Ctrl* host, hipStream_t st);

}  // namespace pint
