// Level loop of the convergence study in eps (Section 3.1).
#pragma once

#include <memory>

#include "internal.h"

namespace sp {

struct ContinuationOut {
  std::unique_ptr<Mesh> mesh;  // the last level's mesh when some level refined
  bool converged = true;       // every linear solve met its tolerance
};

// u0 [m][mesh0->n] host; results [nlev]; lambda [nlev][m] and u_final
// [m][last n] nullable (host).
ContinuationOut run_continuation(Mesh* mesh0, const sp_params& prm, int m, const double* u0,
                                 int nlev, const sp_level* levels, ProjectFn project, void* ctx,
                                 sp_level_result* results, double* lambda, double* u_final);

}  // namespace sp
