// Library-internal entry points shared by the C ABI (pint_api.hip) and the
// serving loop (pint_server.hip): non-blocking pieces of one solve.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "pint.h"
#include "pint_kernels.hpp"

namespace pint {

struct PlanOpts {
  void* d_tables = nullptr;     // device memory for the tables (nullptr: the plan allocates)
  hipStream_t stream = nullptr; // stream of the asynchronous table copy into d_tables
  bool host_mirror = true;      // allocate the plan's own pinned status mirror
  bool defer_tables = false;    // build host tables only; plan_bind_tables uploads them later
};

// Validated plan creation with placement options.
int plan_create_ex(const pint_problem* p, const PlanOpts& opts, pint_plan** out);
// Place the plan's tables in caller-owned device memory d_mem (>= the plan's
// table bytes), copying them asynchronously on st when copy is true.
int plan_bind_tables(pint_plan* pl, void* d_mem, hipStream_t st, bool copy);
// Bytes of the plan's device table block (depends on N and N_t only).
size_t plan_table_bytes(const pint_problem* p);
size_t plan_workspace_bytes(const pint_plan* pl);
int plan_max_iter(const pint_plan* pl);
int plan_nt(const pint_plan* pl);
int plan_ns(const pint_plan* pl);

// Enqueue the initialization of a solve (control record reset, first c_bar)
// on `st`; `host` receives the status mirror written by the control kernel.
int solve_begin(pint_plan* pl, const double* d_u0, double* d_U, void* d_work, size_t work_bytes, hipStream_t st,
                Ctrl* host);
// Enqueue outer iteration `it` (0-based) of that solve.  Iterations after the
// stop flag is set return at once on the device.
int solve_enqueue(pint_plan* pl, const double* d_u0, double* d_U, void* d_work, size_t work_bytes, hipStream_t st,
                  Ctrl* host, int it);
// Status of a finished solve from its mirror; fills rep when non-null.
int solve_status(const pint_plan* pl, const Ctrl& c, pint_report* rep);

}  // namespace pint
