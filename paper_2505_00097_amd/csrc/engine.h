// engine.h -- advancing an ensemble of independent grids together.
//
// The engine owns a device work description (job table + per-variant (job,
// tile) lists + (job, ghost chunk) list, uploaded as one blob) and a cache of
// instantiated hipGraphs, one per step count, each replaying
// steps x 4 stages x [batched RHS kernel per kernel variant, batched ghost
// kernel]. The graphs read the blob at run time, so a changed job set only
// needs a new upload, not a new graph. Tile shapes are chosen per size class
// (coordinate family + interior extents) by timing candidates on the jobs
// themselves; choices persist in a small JSON cache file.
#pragma once

#include <initializer_list>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "bhah_internal.h"

namespace bhah {

// BHAH_OK, or BHAH_EINVAL if any of the (possibly null) arrays is not aligned
// to 8 bytes (a double)
int check_aligned(const char* who, std::initializer_list<const void*> ptrs);

struct EngineJob {
  const bhah_grid* g;
  double* y;
  double* ws;
  double dt;
  // steps this job takes in the next step() call (-1: all of them); a job
  // with fewer steps than the call idles through the rest, its state left
  // after its own last step with every ghost valid
  long long limit = -1;
  bool operator==(const EngineJob& o) const { return g == o.g && y == o.y && ws == o.ws && dt == o.dt; }
};

using SizeClass = std::tuple<int, int, int, int>;  // coord, N0, N1, N2

// tile shapes worth timing for a size class (extent 1 along phi)
std::vector<TileCfg> tile_candidates(const SizeClass& c);

class Engine {
 public:
  Engine(const bhah_gauge_params& gp, const char* cache_path);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  // Replace the job set (takes effect at the next step). Returns a status.
  int set_jobs(const std::vector<EngineJob>& jobs);
  // Advance every job by nsteps steps of the integrator on stream s
  // (asynchronous), job j by min(nsteps, its limit) of them.
  int step(int nsteps, hipStream_t s);
  void set_graph_steps(int S) { graph_steps_ = S < 1 ? 1 : S; }
  // BHAH_RK4 or BHAH_SSPRK3 (the stage arguments and graphs are rebuilt)
  void set_integrator(int k) {
    if (k != integrator_) {
      drop_graphs();
      dirty_ = true;
    }
    integrator_ = k;
  }
  int integrator() const { return integrator_; }
  // persistent blocks of the right-hand-side kernel per compute unit;
  // 0 launches one block per tile instead
  void set_blocks_per_cu(int n) {
    if (n != blocks_per_cu_) drop_graphs();
    blocks_per_cu_ = n < 0 ? 0 : n;
    rhs_blocks_ = 0;
  }

  // Launch tuning: graph steps per captured graph and persistent blocks
  // per CU of the right-hand-side kernel. Off by default; when on, the
  // first step() on a job set not seen before times every candidate pair
  // on copies of the jobs' states (the caller's states are not touched; the
  // results do not depend on either choice) and keeps the fastest, ties
  // within 2% going to the default (10, 4). Choices persist per job-set
  // signature (the multiset of size classes) in the tile cache file.
  void set_launch_tuning(bool on) { tune_launch_ = on; }
  struct LaunchTune {
    int graph_steps = 0, blocks_per_cu = 0;
    double us_per_step = 0.0, default_us_per_step = 0.0, seconds = 0.0;
    int candidates = 0;
    bool from_cache = false;
  };
  const LaunchTune& launch_tune() const { return last_tune_; }

  int n_jobs() const { return (int)jobs_.size(); }
  int n_tiles() const { return n_tiles_; }
  int n_chunks() const { return n_chunks_; }
  int graph_steps() const { return graph_steps_; }
  int blocks_per_cu() const { return blocks_per_cu_; }
  int rhs_blocks() const { return rhs_blocks_; }
  int n_classes_tuned() const { return (int)tuned_.size(); }
  double tune_seconds() const { return tune_seconds_; }
  TileCfg tile_of_class(const SizeClass& c) const;

 private:
  int ensure_device(hipStream_t s);
  int tune_missing(hipStream_t s);
  int time_class(const SizeClass& c, const TileCfg& cfg, hipStream_t s, double* us);
  void build_blob(const std::vector<TileCfg>& cfg, const std::vector<int>& only, int repeat = 1);
  int upload(hipStream_t s);
  int tune_launch(hipStream_t s);
  std::string launch_signature() const;
  // per-job active step counts of one graph launch covering steps
  // [first, first + k) of a step() call, copied to the device blob
  int upload_counts(long long first, int k, hipStream_t s);
  int capture(int nsteps, hipStream_t s, hipGraphExec_t* out);
  void drop_graphs();
  void load_cache();
  void save_cache();

  bhah_gauge_params gp_;
  std::string cache_path_;
  std::string arch_;
  std::vector<EngineJob> jobs_;
  bool dirty_ = true;
  std::map<SizeClass, TileCfg> tuned_;
  std::map<SizeClass, double> tuned_us_;
  double tune_seconds_ = 0.0;
  bool tune_launch_ = false;
  LaunchTune last_tune_{};
  std::map<std::string, std::pair<int, int>> launch_cache_;  // signature -> (graph steps, blocks per CU)
  std::map<std::string, double> launch_us_;

  // host blob (pinned) and its device copy
  char* h_blob_ = nullptr;
  char* d_blob_ = nullptr;
  size_t cap_bytes_ = 0;
  size_t blob_bytes_ = 0;
  int cap_jobs_ = 0, cap_tiles_ = 0, cap_chunks_ = 0;
  hipEvent_t upload_done_ = nullptr;
  // pinned ring of per-launch active step counts (kRing slots of cap_jobs_
  // ints), each slot reused only after its copy has completed
  static constexpr int kRing = 8;
  int* h_counts_ = nullptr;
  hipEvent_t counts_done_[kRing] = {};
  int counts_slot_ = 0;
  int n_tiles_ = 0, n_chunks_ = 0;
  // kernel variants with tiles in some blob (entry NVAR: radiation points)
  bool fam_present_[NVAR + 1] = {};
  bool fam_in_graphs_[NVAR + 1] = {};  // ... and in the captured graphs
  // the ghost lists refilled after a stage (gh[0]: ghosts with an interior
  // phi index, gh[1]: all) and the radiation points of job j: a
  // radiation-boundary grid refills only its inner ghosts (one-hop copies)
  // and evolves its outer points
  struct JobLists {
    GhostDev gh[2];
    RadDev rad;
  };
  JobLists lists_of(int j) const {
    const bhah_grid* g = jobs_[j].g;
    if (g->params.bc_kind == BHAH_BC_RADIATION) return JobLists{{g->ghost_inner_stage, g->ghost_inner}, g->rad};
    return JobLists{{g->ghost_stage, g->ghost}, RadDev{}};
  }

  int rhs_blocks_ = 0, ghost_blocks_ = 0;
  int blocks_per_cu_ = 4;
  int n_cus_ = 0;
  int rhs_grid() const;
  int graph_steps_ = 10;
  int integrator_ = BHAH_RK4;
  std::map<int, hipGraphExec_t> graphs_;
  hipStream_t cap_stream_ = nullptr;
};

}  // namespace bhah
