// batch.cpp -- the bhah_batch_* entry points over the ensemble engine.
#include <new>
#include <vector>

#include "engine.h"

struct bhah_batch {
  std::vector<const bhah_grid*> grids;
  bhah::Engine engine;
  std::vector<int> slot;  // job index in the engine -> grid index, last step
  bhah_batch(const bhah_gauge_params& gp, const char* path) : engine(gp, path) {}
};

extern "C" {

int bhah_batch_create(const bhah_grid* const* grids, int n, const bhah_gauge_params* gp,
                      const char* tune_cache_path, bhah_batch** out) {
  if (!grids || n <= 0 || !gp || !out) return bhah::fail(BHAH_EINVAL, "bhah_batch_create: bad argument");
  if (int rc = bhah::check_gauge(gp, "bhah_batch_create")) return rc;
  for (int j = 0; j < n; j++) {
    if (!grids[j]) return bhah::fail(BHAH_EINVAL, "bhah_batch_create: NULL grid");
  }
  bhah_batch* b = new (std::nothrow) bhah_batch(*gp, tune_cache_path);
  if (!b) return bhah::fail(BHAH_ENOMEM, "bhah_batch_create: host allocation failed");
  b->grids.assign(grids, grids + n);
  *out = b;
  return BHAH_OK;
}

int bhah_batch_step(bhah_batch* b, double* const* y, double* const* ws, const double* host_dt,
                    const unsigned char* host_active, int nsteps, void* stream) {
  if (!b || !y || !ws || !host_dt) return bhah::fail(BHAH_EINVAL, "bhah_batch_step: NULL argument");
  if (nsteps < 0) return bhah::fail(BHAH_EINVAL, "bhah_batch_step: nsteps < 0");
  std::vector<bhah::EngineJob> jobs;
  b->slot.clear();
  for (size_t j = 0; j < b->grids.size(); j++) {
    if (host_active && !host_active[j]) continue;
    if (!y[j] || !ws[j]) return bhah::fail(BHAH_EINVAL, "bhah_batch_step: NULL state or workspace");
    if (int rc = bhah::check_aligned("bhah_batch_step", {y[j], ws[j]})) return rc;
    if (y[j] == ws[j]) return bhah::fail(BHAH_EINVAL, "bhah_batch_step: workspace aliases state");
    jobs.push_back(bhah::EngineJob{b->grids[j], y[j], ws[j], host_dt[j]});
    b->slot.push_back((int)j);
  }
  int rc = b->engine.set_jobs(jobs);
  if (rc) return rc;
  return b->engine.step(nsteps, (hipStream_t)stream);
}

int bhah_batch_set_graph_steps(bhah_batch* b, int steps) {
  if (!b || steps < 1) return bhah::fail(BHAH_EINVAL, "bhah_batch_set_graph_steps: bad argument");
  b->engine.set_graph_steps(steps);
  return BHAH_OK;
}

int bhah_batch_set_integrator(bhah_batch* b, int integrator) {
  if (!b || (integrator != BHAH_RK4 && integrator != BHAH_SSPRK3))
    return bhah::fail(BHAH_EINVAL, "bhah_batch_set_integrator: need a batch and BHAH_RK4 or BHAH_SSPRK3");
  b->engine.set_integrator(integrator);
  return BHAH_OK;
}

int bhah_batch_set_blocks_per_cu(bhah_batch* b, int blocks_per_cu) {
  if (!b || blocks_per_cu < 0) return bhah::fail(BHAH_EINVAL, "bhah_batch_set_blocks_per_cu: bad argument");
  b->engine.set_blocks_per_cu(blocks_per_cu);
  return BHAH_OK;
}

int bhah_batch_get_info(const bhah_batch* b, bhah_batch_info* info) {
  if (!b || !info) return bhah::fail(BHAH_EINVAL, "bhah_batch_get_info: NULL argument");
  info->n_active = b->engine.n_jobs();
  info->n_tiles = b->engine.n_tiles();
  info->n_chunks = b->engine.n_chunks();
  info->graph_steps = b->engine.graph_steps();
  info->rhs_blocks = b->engine.rhs_blocks();
  info->n_classes_tuned = b->engine.n_classes_tuned();
  info->tune_seconds = b->engine.tune_seconds();
  info->blocks_per_cu = b->engine.blocks_per_cu();
  const bhah::Engine::LaunchTune& t = b->engine.launch_tune();
  info->launch_us_per_step = t.us_per_step;
  info->launch_default_us_per_step = t.default_us_per_step;
  info->launch_tune_seconds = t.seconds;
  info->launch_candidates = t.candidates;
  info->launch_from_cache = t.from_cache ? 1 : 0;
  return BHAH_OK;
}

int bhah_batch_set_launch_tuning(bhah_batch* b, int on) {
  if (!b) return bhah::fail(BHAH_EINVAL, "bhah_batch_set_launch_tuning: NULL batch");
  b->engine.set_launch_tuning(on != 0);
  return BHAH_OK;
}

int bhah_batch_get_tile(const bhah_batch* b, int j, int* lx, int* ly, int* band) {
  if (!b || j < 0 || j >= (int)b->grids.size()) return bhah::fail(BHAH_EINVAL, "bhah_batch_get_tile: bad job");
  const bhah_grid* g = b->grids[j];
  const bhah::TileCfg c =
      b->engine.tile_of_class(bhah::SizeClass{g->params.coord, g->params.N[0], g->params.N[1], g->params.N[2]});
  if (lx) *lx = c.lx;
  if (ly) *ly = c.ly;
  if (band) *band = c.band;
  return BHAH_OK;
}

void bhah_batch_destroy(bhah_batch* b) { delete b; }

}  // extern "C"
