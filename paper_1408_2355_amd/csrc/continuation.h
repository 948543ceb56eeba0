// Level loop of the convergence study in eps (Section 3.1).
#pragma once

#include <memory>

#include "internal.h"

namespace sp {

struct ContinuationOut {
  std::unique_ptr<Mesh> mesh;  // the last level's mesh when some level refined
  bool converged = true;       // every linear solve met its tolerance
};

// nres restarts of m components; u0 [nres * m][mesh0->n] host; results
// [nlev][nres]; lambda [nlev][nres * m] and u_final [nres * m][last n]
// nullable (host).
ContinuationOut run_continuation(Mesh* mesh0, const sp_params& prm, int nres, int m,
                                 const double* u0, int nlev, const sp_level* levels,
                                 ProjectFn project, void* ctx, sp_level_result* results,
                                 double* lambda, double* u_final, sp_level_fn on_level,
                                 void* level_ctx);

}  // namespace sp
