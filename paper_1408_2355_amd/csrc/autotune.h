// Tiling autotuner cache.  A tiling of the row-parallel kernels is chosen by
// timing the CG matrix product for a set of candidate (lanes per row, passes
// per chunk, workgroups per XCD range) on the first solver of a given
// (mesh size, ELL width, column count, precision, device); the winner is kept
// in a process-wide table and, when SEGPART_TUNE_CACHE names a file, in that
// JSON file as well (read at first use, rewritten after each new entry).
// SEGPART_AUTOTUNE=0/1 switches the search off/on (default: on for batches of
// at least 2^22 vertex-column values), SEGPART_TUNE_VERBOSE prints the
// timings, SEGPART_SEPS_KERNEL=staged|direct|lanes forces the S_eps element kernel,
// SEGPART_INNER_FLOOR=f (0 < f < 1, default 0.9) sets where a float32 inner
// solve stops relative to the outer target (f x cg_rtol ||b||), and
// SEGPART_SMALL=0 keeps small batches on the multi-kernel path.
#pragma once

#include <string>

namespace sp {

struct TuneChoice {
  int tg_cap = 64;
  int passes = 1;
  int nper_cap = 256;
  double us = 0.0;  // measured time of one matrix product
};

bool tune_lookup(const std::string& key, TuneChoice* out);
void tune_store(const std::string& key, const TuneChoice& c);
// 1 = tune, 0 = default tiling; from SEGPART_AUTOTUNE if set, else `dflt`.
bool tune_enabled(bool dflt);

}  // namespace sp
