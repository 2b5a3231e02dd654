// Autotuner of the scheduling knobs: the cell side of the cell lists, the
// cell size from which the pair search works a cell with whole waves, and
// the number of PGD steps per captured graph.  None of them changes a
// result (cells are never smaller than r_v, the pair sets are sorted before
// use, the union-find roots and the forest are unique), only the time: the
// tuner runs the caller's jobs under each candidate and keeps the fastest.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "host.hpp"

namespace pcc {
namespace {

constexpr int kCellPct[] = {100, 125, 150, 200};
constexpr int kDense[] = {16, 32, 64, 128};
constexpr int kGraph[] = {4, 8, 16, 32};

// One correction of the jobs (outputs discarded).  Returns the wall time of
// the call, or with pair_stages the device time of the stages the cell and
// pair knobs act on (cell build, pair pass, labels, selection, CSR).  Throws
// on a job error so that the tuner does not pick a setting that failed.
double time_call(Context &C, std::vector<pcc_job> &jobs, hipStream_t s, bool pair_stages) {
  std::vector<pcc_job_result> res(jobs.size());
  const auto t0 = std::chrono::steady_clock::now();
  run_batch(C, jobs.data(), (int)jobs.size(), res.data(), s, false);
  PCC_HIP(hipStreamSynchronize(s));
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (auto &r : res)
    if (r.status < 0) throw Error(r.status, "a job failed during autotuning");
  if (!pair_stages) return ms;
  for (auto &r : res)
    if (r.status >= 0) {
      const double *t = r.stats.t_stage_ms;
      return t[1] + t[2] + t[3] + t[4] + t[5];
    }
  return ms;
}

}  // namespace

void autotune(Context &C, const pcc_job *in, int njobs, hipStream_t s, int32_t flags,
              pcc_tune_report &rep) {
  std::memset(&rep, 0, sizeof rep);
  std::vector<pcc_job> jobs(in, in + njobs);
  for (auto &j : jobs) std::memset(&j.out, 0, sizeof j.out);  // nothing is written
  const bool kt = C.kt.on;
  const int pct0 = C.cell_pct, dense0 = C.dense_cell, graph0 = C.graph_iters;
  C.kt.on = false;
  auto record = [&](int kind, double ms) {
    if (rep.n_trials >= PCC_TUNE_MAX_TRIALS) return;
    const int t = rep.n_trials++;
    rep.trial_kind[t] = kind;
    rep.trial_cell_pct[t] = C.cell_pct;
    rep.trial_dense_cell[t] = C.dense_cell;
    rep.trial_graph_iters[t] = C.graph_iters;
    rep.trial_ms[t] = ms;
  };
  try {
    // the stages before PGD under every (cell side, dense threshold)
    time_call(C, jobs, s, false);  // warm-up: arena growth, code loading
    double best = 0.0;
    int best_pct = C.cell_pct, best_dense = C.dense_cell;
    bool first = true;
    for (int pct : kCellPct)
      for (int dense : kDense) {
        C.cell_pct = pct;
        C.dense_cell = dense;
        const double ms = time_call(C, jobs, s, true);
        record(0, ms);
        if (first || ms < best) {
          best = ms;
          best_pct = pct;
          best_dense = dense;
          first = false;
        }
      }
    C.cell_pct = best_pct;
    C.dense_cell = best_dense;
    // steps per captured PGD graph, on whole corrections
    if (!(flags & PCC_TUNE_NO_GRAPH)) {
      int best_g = C.graph_iters;
      first = true;
      for (int g : kGraph) {
        C.graph_iters = g;
        const double ms = time_call(C, jobs, s, false);
        record(1, ms);
        if (first || ms < best) {
          best = ms;
          best_g = g;
          first = false;
        }
      }
      C.graph_iters = best_g;
    }
  } catch (...) {
    C.kt.on = kt;
    C.cell_pct = pct0;
    C.dense_cell = dense0;
    C.graph_iters = graph0;
    throw;
  }
  C.kt.on = kt;
  rep.cell_pct = C.cell_pct;
  rep.dense_cell = C.dense_cell;
  rep.graph_iters = C.graph_iters;
}

}  // namespace pcc
