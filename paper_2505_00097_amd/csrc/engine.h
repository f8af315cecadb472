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
  // (asynchronous).
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

  // host blob (pinned) and its device copy
  char* h_blob_ = nullptr;
  char* d_blob_ = nullptr;
  size_t cap_bytes_ = 0;
  size_t blob_bytes_ = 0;
  int cap_jobs_ = 0, cap_tiles_ = 0, cap_chunks_ = 0;
  hipEvent_t upload_done_ = nullptr;
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
