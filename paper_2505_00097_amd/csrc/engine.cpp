// engine.cpp -- ensemble engine: work lists, graph cache and tile autotuner.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <set>

namespace bhah {

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

SizeClass class_of(const bhah_grid* g) {
  return SizeClass{g->params.coord, g->params.N[0], g->params.N[1], g->params.N[2]};
}

struct Layout {
  size_t jobs, counts, tiles, chunks, total;
};

// header | job table | per-job active step counts | tile list | chunk list
Layout layout(int cap_jobs, int cap_tiles, int cap_chunks) {
  Layout L;
  L.jobs = align_up(sizeof(BatchHdr));
  L.counts = L.jobs + align_up(sizeof(BatchJob) * (size_t)cap_jobs);
  L.tiles = L.counts + align_up(sizeof(int) * (size_t)cap_jobs);
  L.chunks = L.tiles + align_up(sizeof(int2) * (size_t)cap_tiles);
  L.total = L.chunks + align_up(sizeof(int2) * (size_t)cap_chunks);
  return L;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// candidate tile configurations for one size class
std::vector<TileCfg> tile_candidates(const SizeClass& c) {
  const int N0 = std::get<1>(c), N1 = std::get<2>(c), N2 = std::get<3>(c);
  std::vector<TileCfg> out;
  for (int lx = 6; lx >= 3; lx--)
    for (int ly = 0; ly <= 3 && lx + ly <= 6; ly++) {
      if (!tile_fits_periodic(std::get<0>(c), TileCfg{lx, ly, 1})) continue;
      if (ly > 0 && (1 << ly) > N1) continue;
      const int ez = 64 >> (lx + ly);
      if (ez > 1 && ez > N2) continue;
      if (lx < 6 && (1 << lx) > 2 * N0) continue;
      const int ty = (N1 + (1 << ly) - 1) >> ly;
      // bands of 4 and 16 tile rows: tiles that run at the same time share
      // stencil planes in the XCD's L2 (16 pays on large 3-D grids). Wider
      // bands first: near-ties go to the walk with the better L2 reuse (on
      // the head-on grid band 1 moves 1.4x the HBM bytes of band 4 at the
      // same speed within noise)
      if (ty > 8) out.push_back(TileCfg{lx, ly, 16});
      if (ty > 1) out.push_back(TileCfg{lx, ly, 4});
      out.push_back(TileCfg{lx, ly, 1});
    }
  return out;
}

Engine::Engine(const bhah_gauge_params& gp, const char* cache_path) : gp_(gp) {
  if (cache_path) cache_path_ = cache_path;
}

Engine::~Engine() {
  drop_graphs();
  if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
  if (upload_done_) (void)hipEventDestroy(upload_done_);
  for (hipEvent_t& e : counts_done_)
    if (e) (void)hipEventDestroy(e);
  if (h_counts_) (void)hipHostFree(h_counts_);
  if (d_blob_) (void)hipFree(d_blob_);
  if (h_blob_) (void)hipHostFree(h_blob_);
}

TileCfg Engine::tile_of_class(const SizeClass& c) const {
  auto it = tuned_.find(c);
  return it == tuned_.end() ? TileCfg{6, 0, BHAH_DEFAULT_BAND} : it->second;
}

int Engine::set_jobs(const std::vector<EngineJob>& jobs) {
  for (const EngineJob& j : jobs) {
    if (!j.g || !j.y || !j.ws) return fail(BHAH_EINVAL, "batch: NULL grid, state or workspace");
    if (j.g->params.coord < 0 || j.g->params.coord > 2) return fail(BHAH_EINVAL, "batch: bad coordinate family");
  }
  if (jobs != jobs_) {
    jobs_ = jobs;
    dirty_ = true;
  } else {
    // the step limits change from call to call without touching the blob
    for (size_t j = 0; j < jobs.size(); j++) jobs_[j].limit = jobs[j].limit;
  }
  return BHAH_OK;
}

// Blocks of the right-hand-side kernel: blocks_per_cu_ per compute unit
// (the kernel runs one wave per SIMD, so 4 fill a CU) striding over the work
// list, or with blocks_per_cu_ == 0 one block per tile of the current
// capacity; always a multiple of the XCD count.
int Engine::rhs_grid() const {
  const long long want = blocks_per_cu_ > 0 ? (long long)blocks_per_cu_ * n_cus_ : (long long)cap_tiles_;
  return (int)std::max<long long>(BHAH_NXCD, (want + BHAH_NXCD - 1) / BHAH_NXCD * BHAH_NXCD);
}

int Engine::ensure_device(hipStream_t s) {
  (void)s;
  if (upload_done_) return BHAH_OK;
  int dev = 0, cus = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if ((rc = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count")))
    return rc;
  hipDeviceProp_t prop;
  if ((rc = check_hip(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties"))) return rc;
  arch_ = prop.gcnArchName;
  const size_t colon = arch_.find(':');
  if (colon != std::string::npos) arch_ = arch_.substr(0, colon);
  n_cus_ = std::max(cus, 1);
  ghost_blocks_ = 2 * n_cus_;  // times NGF / GF_PER gridfunction groups
  if ((rc = check_hip(hipEventCreateWithFlags(&upload_done_, hipEventDisableTiming), "hipEventCreate"))) return rc;
  for (hipEvent_t& e : counts_done_)
    if ((rc = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate"))) return rc;
  if ((rc = check_hip(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking), "hipStreamCreate"))) return rc;
  load_cache();
  return BHAH_OK;
}

void Engine::drop_graphs() {
  for (auto& kv : graphs_) (void)hipGraphExecDestroy(kv.second);
  graphs_.clear();
  for (int f = 0; f <= NVAR; f++) fam_in_graphs_[f] = false;
}

// Fill the host blob: header, job table (all jobs) and work lists of the
// jobs listed in `only` (all jobs if empty), with tile configuration cfg[j],
// the tile list repeated `repeat` times (timing only: repeated tiles store
// identical values). Grows the buffers if needed (dropping graphs, whose
// arguments point into the old device buffer).
void Engine::build_blob(const std::vector<TileCfg>& cfg, const std::vector<int>& only, int repeat) {
  std::vector<int> sel = only;
  if (sel.empty())
    for (int j = 0; j < (int)jobs_.size(); j++) sel.push_back(j);
  std::vector<TileMap> maps(jobs_.size());
  int nt = 0, nc = 0;
  for (int j = 0; j < (int)jobs_.size(); j++)
    maps[j] = make_tilemap(jobs_[j].g->dev, cfg[j].lx, cfg[j].ly, cfg[j].band);
  for (int j : sel) {
    nt += maps[j].ntiles * repeat;
    const JobLists l = lists_of(j);
    nc += (l.gh[0].n_ghost + 255) / 256 + (l.gh[1].n_ghost + 255) / 256 + (l.rad.n + 255) / 256;
  }
  // the previous upload must have left the pinned buffer before it is reused
  if (upload_done_) (void)hipEventSynchronize(upload_done_);
  if ((int)jobs_.size() > cap_jobs_ || nt > cap_tiles_ || nc > cap_chunks_) {
    (void)hipDeviceSynchronize();
    drop_graphs();
    if (d_blob_) (void)hipFree(d_blob_);
    if (h_blob_) (void)hipHostFree(h_blob_);
    if (h_counts_) (void)hipHostFree(h_counts_);
    d_blob_ = h_blob_ = nullptr;
    h_counts_ = nullptr;
    cap_jobs_ = std::max<int>(cap_jobs_, (int)jobs_.size() * 3 / 2 + 1);
    cap_tiles_ = std::max(cap_tiles_, nt * 3 / 2 + 64);
    cap_chunks_ = std::max(cap_chunks_, nc * 3 / 2 + 64);
    const Layout L = layout(cap_jobs_, cap_tiles_, cap_chunks_);
    cap_bytes_ = L.total;
    if (hipMalloc((void**)&d_blob_, cap_bytes_) != hipSuccess ||
        hipHostMalloc((void**)&h_blob_, cap_bytes_, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_counts_, sizeof(int) * kRing * (size_t)cap_jobs_, hipHostMallocDefault) !=
            hipSuccess) {
      set_error("batch: cannot allocate the work description");
      cap_bytes_ = 0;
      cap_jobs_ = cap_tiles_ = cap_chunks_ = 0;
      return;
    }
  }
  const Layout L = layout(cap_jobs_, cap_tiles_, cap_chunks_);
  BatchHdr* hdr = (BatchHdr*)h_blob_;
  BatchJob* J = (BatchJob*)(h_blob_ + L.jobs);
  int2* tiles = (int2*)(h_blob_ + L.tiles);
  int2* chunks = (int2*)(h_blob_ + L.chunks);
  std::memset(hdr, 0, sizeof(BatchHdr));
  for (int j = 0; j < (int)jobs_.size(); j++) {
    const EngineJob& e = jobs_[j];
    BatchJob& b = J[j];
    b.G = e.g->dev;
    const JobLists l = lists_of(j);
    b.gh[0] = l.gh[0];
    b.gh[1] = l.gh[1];
    b.rad = l.rad;
    b.T = maps[j];
    const double* in[4] = {nullptr, nullptr, nullptr, nullptr};
    double* gd[4] = {nullptr, nullptr, nullptr, nullptr};
    if (integrator_ == BHAH_SSPRK3) {
      ssprk3_stages(e.dt, e.y, e.ws, e.g->info.state_doubles, b.st, in, gd);
      b.st[3] = StageArgs{};
    } else {
      rk4_stages(e.dt, e.y, e.ws, e.g->info.state_doubles, b.st, in, gd);
    }
    for (int k = 0; k < 4; k++) {
      b.in[k] = in[k];
      b.gdst[k] = gd[k];
    }
    b.st[4] = StageArgs{e.ws, nullptr, nullptr, 0.0, nullptr, nullptr, 0.0};
    b.in[4] = e.y;
    b.gdst[4] = nullptr;
  }
  int pos = 0;
  for (int f = 0; f < NVAR; f++) {
    hdr->tile_off[f] = pos;
    for (int r = 0; r < repeat; r++)
      for (int j : sel) {
        const GridDev& G = jobs_[j].g->dev;
        if (rhs_variant(G.coord, G.N1, G.N2, G.ng) != f) continue;
        for (int t = 0; t < maps[j].ntiles; t++) tiles[pos++] = int2{j, t};
      }
    hdr->n_tiles[f] = pos - hdr->tile_off[f];
    fam_present_[f] = hdr->n_tiles[f] > 0 || fam_present_[f];
  }
  int cpos = 0;
  for (int w = 0; w < 3; w++) {
    hdr->chunk_off[w] = cpos;
    for (int j : sel) {
      const JobLists l = lists_of(j);
      const int pts = w < 2 ? l.gh[w].n_ghost : l.rad.n;
      const int n = (pts + 255) / 256;
      for (int c = 0; c < n; c++) chunks[cpos++] = int2{j, c};
    }
    hdr->n_chunks[w] = cpos - hdr->chunk_off[w];
  }
  fam_present_[NVAR] = hdr->n_chunks[2] > 0 || fam_present_[NVAR];
  n_tiles_ = pos;
  n_chunks_ = cpos;
  blob_bytes_ = (size_t)(L.chunks + sizeof(int2) * (size_t)cpos);
}

int Engine::upload(hipStream_t s) {
  if (!d_blob_) return fail(BHAH_ENOMEM, "batch: no work description buffer");
  int rc = check_hip(hipMemcpyAsync(d_blob_, h_blob_, blob_bytes_, hipMemcpyHostToDevice, s), "batch upload");
  if (rc) return rc;
  return check_hip(hipEventRecord(upload_done_, s), "hipEventRecord");
}

int Engine::upload_counts(long long first, int k, hipStream_t s) {
  if (!d_blob_ || !h_counts_) return fail(BHAH_ENOMEM, "batch: no work description buffer");
  const int slot = counts_slot_;
  counts_slot_ = (counts_slot_ + 1) % kRing;
  int rc = check_hip(hipEventSynchronize(counts_done_[slot]), "batch counts slot");
  if (rc) return rc;
  int* h = h_counts_ + (size_t)slot * cap_jobs_;
  for (size_t j = 0; j < jobs_.size(); j++) {
    const long long lim = jobs_[j].limit < 0 ? first + k : jobs_[j].limit;
    h[j] = (int)std::max<long long>(0, std::min<long long>(k, lim - first));
  }
  const Layout L = layout(cap_jobs_, cap_tiles_, cap_chunks_);
  rc = check_hip(hipMemcpyAsync(d_blob_ + L.counts, h, sizeof(int) * jobs_.size(), hipMemcpyHostToDevice, s),
                 "batch counts upload");
  if (rc) return rc;
  return check_hip(hipEventRecord(counts_done_[slot], s), "hipEventRecord");
}

int Engine::time_class(const SizeClass& c, const TileCfg& cfg, hipStream_t s, double* us) {
  std::vector<int> only;
  std::vector<TileCfg> cfgs(jobs_.size(), TileCfg{6, 0, 1});
  long long tiles = 0;
  for (int j = 0; j < (int)jobs_.size(); j++)
    if (class_of(jobs_[j].g) == c) {
      only.push_back(j);
      cfgs[j] = cfg;
      tiles += make_tilemap(jobs_[j].g->dev, cfg.lx, cfg.ly, cfg.band).ntiles;
    }
  // time the class at full occupancy: repeat its tiles until every
  // persistent block slot sees several
  const long long target = 16LL * n_cus_;
  const int repeat = (int)std::max<long long>(1, (target + tiles - 1) / std::max<long long>(tiles, 1));
  build_blob(cfgs, only, repeat);
  int rc = upload(s);
  if (rc) return rc;
  const Layout L = layout(cap_jobs_, cap_tiles_, cap_chunks_);
  const BatchJob* dj = (const BatchJob*)(d_blob_ + L.jobs);
  const BatchHdr* dh = (const BatchHdr*)d_blob_;
  const int2* dt = (const int2*)(d_blob_ + L.tiles);
  // the kernel variants of the class's jobs (4th- and 8th-order grids of one
  // shape share the class)
  bool used[NVAR] = {};
  for (int j : only) {
    const GridDev& G = jobs_[j].g->dev;
    used[rhs_variant(G.coord, G.N1, G.N2, G.ng)] = true;
  }
  hipEvent_t e0, e1;
  if ((rc = check_hip(hipEventCreate(&e0), "hipEventCreate"))) return rc;
  if ((rc = check_hip(hipEventCreate(&e1), "hipEventCreate"))) { (void)hipEventDestroy(e0); return rc; }
  const int reps = 3;
  const int blocks = rhs_grid();
  for (int v = 0; v < NVAR; v++)
    if (used[v]) launch_rhs_batch(v, dj, dh, dt, 4, nullptr, 0, gauge_of(gp_), false, blocks, s);
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; r++)
    for (int v = 0; v < NVAR; v++)
      if (used[v]) launch_rhs_batch(v, dj, dh, dt, 4, nullptr, 0, gauge_of(gp_), false, blocks, s);
  (void)hipEventRecord(e1, s);
  rc = check_hip(hipEventSynchronize(e1), "tile timing");
  float ms = 0.f;
  if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us = 1e3 * ms / reps / repeat;
  return rc;
}

int Engine::tune_missing(hipStream_t s) {
  std::set<SizeClass> todo;
  for (const EngineJob& j : jobs_)
    if (!tuned_.count(class_of(j.g))) todo.insert(class_of(j.g));
  if (todo.empty()) return BHAH_OK;
  const double t0 = now_s();
  for (const SizeClass& c : todo) {
    double best = 1e300;
    TileCfg bc{6, 0, 1};
    for (const TileCfg& cfg : tile_candidates(c)) {
      double us = 0.0;
      const int rc = time_class(c, cfg, s, &us);
      if (rc) return rc;
      if (us < best) {
        best = us;
        bc = cfg;
      }
    }
    tuned_[c] = bc;
    tuned_us_[c] = best;
  }
  tune_seconds_ += now_s() - t0;
  dirty_ = true;
  save_cache();
  return BHAH_OK;
}

int Engine::capture(int nsteps, hipStream_t s, hipGraphExec_t* out) {
  (void)s;
  const Layout L = layout(cap_jobs_, cap_tiles_, cap_chunks_);
  const BatchJob* dj = (const BatchJob*)(d_blob_ + L.jobs);
  const BatchHdr* dh = (const BatchHdr*)d_blob_;
  const int2* dt = (const int2*)(d_blob_ + L.tiles);
  const int2* dc = (const int2*)(d_blob_ + L.chunks);
  const int* dn = (const int*)(d_blob_ + L.counts);
  rhs_blocks_ = rhs_grid();
  int rc = check_hip(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal), "graph capture");
  if (rc) return rc;
  // Step k of the graph runs the jobs with more than k active steps in this
  // launch (counts, uploaded before each launch). The stencils never read
  // phi ghost planes (they wrap phi onto the interior), so within a job's
  // steps only the ghosts with an interior phi index are filled; the last
  // stage of its last active step fills all of them.
  const int nst = integrator_ == BHAH_SSPRK3 ? 3 : 4;
  for (int k = 0; k < nsteps; k++)
    for (int stage = 0; stage < nst; stage++) {
      for (int f = 0; f < NVAR; f++)
        if (fam_present_[f])
          launch_rhs_batch(f, dj, dh, dt, stage, dn, k, gauge_of(gp_), integrator_ == BHAH_SSPRK3, rhs_blocks_,
                           cap_stream_);
      // outer points of radiation-boundary jobs, before their inner ghosts are copied
      if (fam_present_[NVAR]) launch_radiation_batch(dj, dh, dc, stage, dn, k, ghost_blocks_, cap_stream_);
      launch_ghosts_batch(dj, dh, dc, stage, dn, k, stage == nst - 1, ghost_blocks_, cap_stream_);
    }
  hipGraph_t graph = nullptr;
  const hipError_t le = hipGetLastError();
  rc = check_hip(hipStreamEndCapture(cap_stream_, &graph), "graph capture end");
  if (!rc && le != hipSuccess) rc = check_hip(le, "graph capture launch");
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  rc = check_hip(hipGraphInstantiate(out, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  (void)hipGraphDestroy(graph);
  for (int f = 0; f <= NVAR; f++) fam_in_graphs_[f] = fam_present_[f];
  return rc;
}

int Engine::step(int nsteps, hipStream_t s) {
  if (nsteps < 0) return fail(BHAH_EINVAL, "batch: nsteps < 0");
  if (jobs_.empty() || nsteps == 0) return BHAH_OK;
  int rc = ensure_device(s);
  if (rc) return rc;
  if ((rc = tune_missing(s))) return rc;
  if (dirty_) {
    std::vector<TileCfg> cfg;
    for (const EngineJob& j : jobs_) cfg.push_back(tile_of_class(class_of(j.g)));
    build_blob(cfg, {});
    if ((rc = upload(s))) return rc;
    dirty_ = false;
  }
  if (tune_launch_ && (rc = tune_launch(s))) return rc;
  for (int f = 0; f <= NVAR; f++)
    if (fam_present_[f] && !fam_in_graphs_[f]) drop_graphs();
  // jobs that take fewer steps than the call idle through the rest: launch
  // graphs only while some job still has steps to take
  long long most = 0;
  for (const EngineJob& j : jobs_) most = std::max<long long>(most, j.limit < 0 ? nsteps : std::min<long long>(nsteps, j.limit));
  long long first = 0;
  while (first < most) {
    const int k = (int)std::min<long long>(most - first, graph_steps_);
    auto it = graphs_.find(k);
    if (it == graphs_.end()) {
      hipGraphExec_t ex = nullptr;
      if ((rc = capture(k, s, &ex))) return rc;
      it = graphs_.emplace(k, ex).first;
    }
    if ((rc = upload_counts(first, k, s))) return rc;
    if ((rc = check_hip(hipGraphLaunch(it->second, s), "hipGraphLaunch"))) return rc;
    first += k;
  }
  return BHAH_OK;
}

std::string Engine::launch_signature() const {
  std::map<std::string, int> count;
  for (const EngineJob& j : jobs_) {
    const bhah_grid_params& p = j.g->params;
    char b[96];
    std::snprintf(b, sizeof b, "%d:%dx%dx%d:%d:%d", p.coord, p.N[0], p.N[1], p.N[2], p.nghosts, p.bc_kind);
    count[b]++;
  }
  std::string full;
  for (auto& kv : count) full += std::to_string(kv.second) + "*" + kv.first + " ";
  unsigned long long h = 1469598103934665603ULL;  // FNV-1a, stable across runs and builds
  for (unsigned char c : full) h = (h ^ c) * 1099511628211ULL;
  char b[96];
  std::snprintf(b, sizeof b, "%s %zu jobs %016llx", integrator_ == BHAH_SSPRK3 ? "ssprk3" : "rk4", jobs_.size(), h);
  return b;
}

int Engine::tune_launch(hipStream_t s) {
  const std::string sig = launch_signature();
  auto hit = launch_cache_.find(sig);
  if (hit != launch_cache_.end()) {
    if (hit->second.first != graph_steps_ || hit->second.second != blocks_per_cu_) {
      set_graph_steps(hit->second.first);
      set_blocks_per_cu(hit->second.second);
      drop_graphs();
    }
    last_tune_.graph_steps = graph_steps_;
    last_tune_.blocks_per_cu = blocks_per_cu_;
    last_tune_.from_cache = true;
    auto u = launch_us_.find(sig);
    last_tune_.us_per_step = u == launch_us_.end() ? 0.0 : u->second;
    return BHAH_OK;
  }
  const double t0 = now_s();
  // copies of the states: the candidates run real steps
  size_t total = 0;
  for (const EngineJob& j : jobs_) total += (size_t)j.g->info.state_doubles;
  double* copies = nullptr;
  if (hipMalloc((void**)&copies, total * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BHAH_ENOMEM, "batch: no device memory for the launch tuning's state copies");
  }
  const std::vector<EngineJob> saved = jobs_;
  size_t off = 0;
  int rc = BHAH_OK;
  for (EngineJob& j : jobs_) {
    const size_t n = (size_t)j.g->info.state_doubles;
    if (!rc) rc = check_hip(hipMemcpyAsync(copies + off, j.y, n * sizeof(double), hipMemcpyDeviceToDevice, s),
                            "launch tuning copy");
    j.y = copies + off;
    j.limit = -1;
    off += n;
  }
  std::vector<TileCfg> cfg;
  for (const EngineJob& j : jobs_) cfg.push_back(tile_of_class(class_of(j.g)));
  if (!rc) {
    build_blob(cfg, {});
    rc = upload(s);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc) rc = check_hip(hipEventCreate(&e0), "hipEventCreate");
  if (!rc) rc = check_hip(hipEventCreate(&e1), "hipEventCreate");
  const int steps_c[3] = {4, 10, 25}, bpc_c[4] = {2, 4, 8, 0};
  int best_s = 10, best_b = 4;
  double best = 1e300, def = 0.0;
  int n_cand = 0;
  for (int a = 0; a < 3 && !rc; a++)
    for (int b = 0; b < 4 && !rc; b++) {
      set_graph_steps(steps_c[a]);
      set_blocks_per_cu(bpc_c[b]);
      drop_graphs();
      hipGraphExec_t ex = nullptr;
      if ((rc = capture(graph_steps_, s, &ex))) break;
      graphs_.emplace(graph_steps_, ex);
      if ((rc = upload_counts(0, graph_steps_, s))) break;
      (void)hipGraphLaunch(ex, s);  // warm-up
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 2; r++) (void)hipGraphLaunch(ex, s);
      (void)hipEventRecord(e1, s);
      if ((rc = check_hip(hipEventSynchronize(e1), "launch tuning"))) break;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double us = 1e3 * ms / (2.0 * graph_steps_);
      n_cand++;
      if (steps_c[a] == 10 && bpc_c[b] == 4) def = us;
      if (us < best) {
        best = us;
        best_s = steps_c[a];
        best_b = bpc_c[b];
      }
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(copies);
  jobs_ = saved;
  dirty_ = true;
  drop_graphs();
  if (rc) return rc;
  if (def > 0.0 && best >= def / 1.02) {  // within 2% of the default: keep it
    best_s = 10;
    best_b = 4;
    best = def;
  }
  set_graph_steps(best_s);
  set_blocks_per_cu(best_b);
  // the tuning blob held the copies: rebuild with the jobs' own states
  build_blob(cfg, {});
  if ((rc = upload(s))) return rc;
  dirty_ = false;
  launch_cache_[sig] = {best_s, best_b};
  launch_us_[sig] = best;
  last_tune_ = LaunchTune{best_s, best_b, best, def, now_s() - t0, n_cand, false};
  save_cache();
  return BHAH_OK;
}

// ---- tile cache: one JSON object per line inside an "entries" array -----
void Engine::load_cache() {
  if (cache_path_.empty()) return;
  FILE* f = std::fopen(cache_path_.c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char arch[64];
    int coord, n0, n1, n2, lx, ly, band;
    double us;
    const char* p = std::strchr(line, '{');
    if (!p) continue;
    {  // a launch-configuration entry
      char sig[96];
      int S, bpc;
      if (std::sscanf(p, "{\"arch\": \"%63[^\"]\", \"launch\": \"%95[^\"]\", \"S\": %d, \"bpc\": %d, \"us\": %lf}",
                      arch, sig, &S, &bpc, &us) == 5) {
        if (arch_ == arch && S >= 1 && bpc >= 0) {
          launch_cache_[sig] = {S, bpc};
          launch_us_[sig] = us;
        }
        continue;
      }
    }
    if (std::sscanf(p, "{\"arch\": \"%63[^\"]\", \"coord\": %d, \"N\": [%d, %d, %d], \"lx\": %d, \"ly\": %d, "
                       "\"band\": %d, \"us\": %lf}",
                    arch, &coord, &n0, &n1, &n2, &lx, &ly, &band, &us) != 9)
      continue;
    if (arch_ != arch) continue;
    if (lx < 0 || ly < 0 || lx + ly > 6 || band < 1) continue;
    if (coord < 0 || coord > 2 || !tile_fits_periodic(coord, TileCfg{lx, ly, band})) continue;
    tuned_[SizeClass{coord, n0, n1, n2}] = TileCfg{lx, ly, band};
    tuned_us_[SizeClass{coord, n0, n1, n2}] = us;
  }
  std::fclose(f);
}

void Engine::save_cache() {
  if (cache_path_.empty()) return;
  // keep entries of other architectures that are in the file
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(cache_path_.c_str(), "r")) {
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
      const char* p = std::strstr(line, "{\"arch\": \"");
      if (!p) continue;
      const std::string a = std::string("{\"arch\": \"") + arch_ + "\"";
      if (std::strncmp(p, a.c_str(), a.size()) == 0) continue;
      std::string l(p);
      while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == ' ')) l.pop_back();
      keep.push_back(l);
    }
    std::fclose(f);
  }
  const std::string tmp = cache_path_ + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\"bhah_tile_cache\": 1, \"entries\": [\n");
  bool first = true;
  for (const std::string& l : keep) {
    std::fprintf(f, "%s%s", first ? "" : ",\n", l.c_str());
    first = false;
  }
  for (const auto& kv : tuned_) {
    const SizeClass& c = kv.first;
    const auto u = tuned_us_.find(c);
    std::fprintf(f,
                 "%s{\"arch\": \"%s\", \"coord\": %d, \"N\": [%d, %d, %d], \"lx\": %d, \"ly\": %d, \"band\": %d, "
                 "\"us\": %.3f}",
                 first ? "" : ",\n", arch_.c_str(), std::get<0>(c), std::get<1>(c), std::get<2>(c),
                 std::get<3>(c), kv.second.lx, kv.second.ly, kv.second.band,
                 u == tuned_us_.end() ? 0.0 : u->second);
    first = false;
  }
  for (const auto& kv : launch_cache_) {
    const auto u = launch_us_.find(kv.first);
    std::fprintf(f, "%s{\"arch\": \"%s\", \"launch\": \"%s\", \"S\": %d, \"bpc\": %d, \"us\": %.3f}",
                 first ? "" : ",\n", arch_.c_str(), kv.first.c_str(), kv.second.first, kv.second.second,
                 u == launch_us_.end() ? 0.0 : u->second);
    first = false;
  }
  std::fprintf(f, "\n]}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), cache_path_.c_str());
}

}  // namespace bhah
