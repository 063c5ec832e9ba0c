// Internal interface between the host runtime and the kernels: argument
// blocks, the device control record and the launcher declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "device_common.hpp"

namespace pint {

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
};

struct ResidArgs {
  const double* u0;
  const double* U;
  double* part;
  const int* done;
  double inv_dt, inv_h2, theta;
  double c1, c1p, c2, c3;
};

struct UpdArgs {
  double* U;
  double* part;
  const int* done;
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
};

struct FinArgs {
  Ctrl* ctrl;
  const double* part;
  int nt, max_iter;
  double dof, rtol;
};

struct InitArgs {
  const double* u0;
  double* U;
  double* part;
  int nt, ns, broadcast;
};

struct DiagArgs {
  const double* U;
  double* mass;
  double* energy;
  int nx, ns, dim;
  double eps2, inv_h2, hd;
};

template <typename T>
hipError_t launch_resid(int dim, int n, const ResidArgs& a, T* S, double* rout, const DctTables<T>& dt, int nt,
                        int mode, hipStream_t st);
template <typename T>
hipError_t launch_update(int dim, int n, const UpdArgs& a, const T* S, double* dout, const DctTables<T>& dt, int nt,
                         int mode, hipStream_t st);
template <typename T>
hipError_t launch_dct(int dim, int n, const T* in, T* out, const DctTables<T>& dt, int nt, bool inv,
                      hipStream_t st);
template <typename T>
hipError_t launch_time(int nt, T* S, const TimeArgs<T>& ta, hipStream_t st);
template <typename T>
hipError_t launch_cast_to(const double* in, T* out, size_t n, hipStream_t st);
template <typename T>
hipError_t launch_cast_from(const T* in, double* out, size_t n, hipStream_t st);
hipError_t launch_finalize(const FinArgs& f, hipStream_t st);
hipError_t launch_init(const InitArgs& a, Ctrl* c, double dof, hipStream_t st);
hipError_t launch_diagnostics(const DiagArgs& a, int nt, hipStream_t st);

}  // namespace pint
