// Shared PGD loop of the served form (iteration-level continuous batching).
//
// Each call the server runs prepares its jobs on its own stream (input
// scan, cells, pairs, selection, CSR, the first PGD step), then hands its
// PGD state to this loop as one group and waits.  The loop owns one stream
// and one captured graph of K steps (a step launch and a finalize launch
// each) over a device table of groups; between two replays it reads which
// groups have no job left, removes them (their calls go on to encode on
// their own streams) and adds the groups that arrived meanwhile.  So a job
// that arrives while others iterate starts iterating at the next replay,
// and a job that converges leaves at the end of the replay in which it did,
// whatever the other jobs do.  The step kernel walks the tiles of every
// group in one launch; each job keeps its own iterates, Adam state,
// counters and stopping test, so its results are those of running it alone.
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "host.hpp"

namespace pcc {

class PgdEngine {
 public:
  PgdEngine(int device, int graph_iters) : device_(device), K_(graph_iters) {
    th_ = std::thread([this] { main(); });
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return ready_; });
    if (!error_.empty()) {
      lk.unlock();
      th_.join();
      throw Error(PCC_E_DEVICE, "shared PGD loop: " + error_);
    }
  }

  ~PgdEngine() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_work_.notify_all();
    if (th_.joinable()) th_.join();
  }

  void run(const PgdBufs &gb, int32_t active) {
    Member m;
    m.b = gb;
    m.active = active;
    m.jobs = gb.njobs;
    m.tiles = gb.ntiles;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!error_.empty()) throw Error(PCC_E_DEVICE, "shared PGD loop: " + error_);
      pending_.push_back(&m);
    }
    cv_work_.notify_all();
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return m.done; });
    if (!m.error.empty()) throw Error(PCC_E_DEVICE, "shared PGD loop: " + m.error);
  }

 private:
  struct Member {
    PgdBufs b;
    int32_t active = 0;  // jobs not done
    int32_t jobs = 0;
    int64_t tiles = 0;
    bool done = false;
    std::string error;
  };

  void fail_all(const std::string &msg) {
    std::lock_guard<std::mutex> lk(mu_);
    error_ = msg;
    for (auto *v : {&pending_, &resident_})
      for (Member *m : *v) {
        m->error = msg;
        m->done = true;
      }
    pending_.clear();
    resident_.clear();
    ready_ = true;
    cv_done_.notify_all();
  }

  void setup() {
    PCC_HIP(hipSetDevice(device_));
    PCC_HIP(hipStreamCreate(&s_));
    PCC_HIP(hipMalloc((void **)&d_tab_, sizeof(PgdGroups)));
    PCC_HIP(hipHostMalloc((void **)&h_tab_, sizeof(PgdGroups), hipHostMallocDefault));
    std::memset(h_tab_, 0, sizeof(PgdGroups));
    PCC_HIP(hipMemcpyAsync(d_tab_, h_tab_, sizeof(PgdGroups), hipMemcpyHostToDevice, s_));
    PCC_HIP(hipStreamSynchronize(s_));
    const int K = std::max(1, std::min(64, K_));
    PCC_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < K; ++k) {
      launch_pgd_step_shared(d_tab_, s_);
      launch_pgd_finalize_shared(d_tab_, s_);
    }
    PCC_HIP(hipStreamEndCapture(s_, &graph_));
    PCC_HIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
  }

  void teardown() {
    if (s_) hipStreamSynchronize(s_);
    if (exec_) hipGraphExecDestroy(exec_);
    if (graph_) hipGraphDestroy(graph_);
    if (d_tab_) hipFree(d_tab_);
    if (h_tab_) hipHostFree(h_tab_);
    if (s_) hipStreamDestroy(s_);
  }

  // the device table of the resident groups (their counts and the address
  // of each group's count slot included)
  void build_table() {
    PgdGroups &T = *h_tab_;
    T.ngroups = (int32_t)resident_.size();
    T.tile_base[0] = 0;
    T.job_base[0] = 0;
    for (size_t g = 0; g < resident_.size(); ++g) {
      Member &m = *resident_[g];
      T.g[g] = m.b;
      T.g[g].n_active = d_tab_->active + g;
      T.active[g] = m.active;
      T.tile_base[g + 1] = T.tile_base[g] + m.tiles;
      T.job_base[g + 1] = T.job_base[g] + m.jobs;
    }
  }

  void main() {
    try {
      setup();
    } catch (const std::exception &e) {
      fail_all(e.what());
      teardown();
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      ready_ = true;
    }
    cv_done_.notify_all();
    try {
      for (;;) {
        {
          std::unique_lock<std::mutex> lk(mu_);
          cv_work_.wait(lk, [&] { return stop_ || !pending_.empty() || !resident_.empty(); });
          if (pending_.empty() && resident_.empty()) break;  // stopping, nothing left
          // arrivals join while the table has room
          int jobs = 0;
          for (Member *m : resident_) jobs += m->jobs;
          size_t k = 0;
          for (; k < pending_.size(); ++k) {
            Member *m = pending_[k];
            if ((int)resident_.size() >= kMaxGroups || jobs + m->jobs > kMaxGroupJobs) break;
            resident_.push_back(m);
            jobs += m->jobs;
          }
          pending_.erase(pending_.begin(), pending_.begin() + k);
        }
        build_table();
        PCC_HIP(hipMemcpyAsync(d_tab_, h_tab_, sizeof(PgdGroups), hipMemcpyHostToDevice, s_));
        PCC_HIP(hipGraphLaunch(exec_, s_));
        PCC_HIP(hipMemcpyAsync(h_tab_->active, d_tab_->active, sizeof(h_tab_->active),
                               hipMemcpyDeviceToHost, s_));
        PCC_HIP(hipStreamSynchronize(s_));
        std::lock_guard<std::mutex> lk(mu_);
        std::vector<Member *> keep;
        for (size_t g = 0; g < resident_.size(); ++g) {
          Member *m = resident_[g];
          m->active = h_tab_->active[g];
          if (m->active <= 0)
            m->done = true;
          else
            keep.push_back(m);
        }
        resident_.swap(keep);
        cv_done_.notify_all();
      }
    } catch (const std::exception &e) {
      fail_all(e.what());
    }
    teardown();
  }

  int device_;
  int K_;
  hipStream_t s_ = nullptr;
  PgdGroups *d_tab_ = nullptr;
  PgdGroups *h_tab_ = nullptr;  // pinned
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::vector<Member *> pending_, resident_;
  bool stop_ = false;
  bool ready_ = false;
  std::string error_;
  std::thread th_;
};

PgdEngine *engine_create(int device, int graph_iters) { return new PgdEngine(device, graph_iters); }

void engine_destroy(PgdEngine *e) { delete e; }

void engine_run(PgdEngine *e, const PgdBufs &gb, int32_t active) { e->run(gb, active); }

}  // namespace pcc
