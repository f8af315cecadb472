// batch.cpp -- ensembles of independent grids (placeholder sequential form,
// superseded by the batched kernels once they land).
#include <vector>

#include "bhah_internal.h"

struct bhah_batch {
  std::vector<const bhah_grid*> grids;
  bhah_gauge_params gp;
};

extern "C" {

int bhah_batch_create(const bhah_grid* const* grids, int n, const bhah_gauge_params* gp,
                      const char* tune_cache_path, bhah_batch** out) {
  (void)tune_cache_path;
  if (!grids || n <= 0 || !gp || !out) return bhah::fail(BHAH_EINVAL, "bhah_batch_create: bad argument");
  bhah_batch* b = new bhah_batch();
  b->grids.assign(grids, grids + n);
  b->gp = *gp;
  *out = b;
  return BHAH_OK;
}

int bhah_batch_step(bhah_batch* b, double* const* y, double* const* ws, const double* host_dt,
                    const unsigned char* host_active, int nsteps, void* stream) {
  if (!b || !y || !ws || !host_dt) return bhah::fail(BHAH_EINVAL, "bhah_batch_step: NULL argument");
  for (int s = 0; s < nsteps; s++)
    for (size_t j = 0; j < b->grids.size(); j++) {
      if (host_active && !host_active[j]) continue;
      const int rc = bhah_rk4_step(b->grids[j], &b->gp, host_dt[j], y[j], ws[j], stream);
      if (rc) return rc;
    }
  return BHAH_OK;
}

void bhah_batch_destroy(bhah_batch* b) { delete b; }

}  // extern "C"
