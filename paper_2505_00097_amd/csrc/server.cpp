// server.cpp -- continuous batching of evolution jobs over the ensemble engine.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "engine.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// grid parameters as a byte key (the struct has no padding holes that the
// caller could leave uninitialised after we copy it field by field)
std::string grid_key(const bhah_grid_params& p) {
  bhah_grid_params c;
  std::memset(&c, 0, sizeof c);
  c.coord = p.coord;
  for (int d = 0; d < 3; d++) {
    c.N[d] = p.N[d];
    c.ampl[d] = p.ampl[d];
    c.sinhw[d] = p.sinhw[d];
  }
  c.nghosts = p.nghosts;
  c.cfl = p.cfl;
  c.bc_kind = p.bc_kind;
  return std::string((const char*)&c, sizeof c);
}

double weighted_percentile(std::vector<std::pair<double, double>> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  double total = 0.0;
  for (auto& x : v) total += x.second;
  const double target = p / 100.0 * total;
  double acc = 0.0;
  for (auto& x : v) {
    acc += x.second;
    if (acc >= target) return x.first;
  }
  return v.back().first;
}

}  // namespace

struct bhah_server {
  struct Job {
    bhah_job_desc d;
    std::string key;
    bhah_grid* g = nullptr;
    double* mem = nullptr;  // state | workspace (4 state copies)
    int state = BHAH_JOB_QUEUED;
    long long done = 0;
    double t_submit = -1, t_admit = -1, t_done = -1;
  };

  bhah_server_params p;
  hipStream_t stream;
  bhah::Engine engine;
  double t0;
  std::map<std::string, bhah_grid*> grids;
  std::map<std::string, std::vector<double*>> free_slabs;
  std::vector<double*> all_slabs;
  double held = 0.0, peak_held = 0.0;
  std::unordered_map<long long, Job> jobs;
  std::deque<long long> queue;
  std::vector<long long> running;
  long long next_id = 1;
  long long n_done = 0;
  long long point_steps = 0;
  double busy = 0.0;
  int peak_running = 0;
  std::vector<std::pair<double, double>> step_ms;  // (latency, job-steps)
  std::vector<std::pair<double, double>> job_s;    // (latency, 1)

  bhah_server(const bhah_server_params& prm, hipStream_t s)
      : p(prm), stream(s), engine(prm.gauge, prm.tune_cache_path), t0(now_s()) {}
  ~bhah_server() {
    (void)hipStreamSynchronize(stream);
    for (double* m : all_slabs) (void)hipFree(m);
    for (auto& kv : grids) bhah_grid_destroy(kv.second);
  }
  double now() const { return now_s() - t0; }
  static double slab_bytes(const bhah_grid* g) { return 4.0 * 8.0 * (double)g->info.state_doubles; }

  int grid_for(Job& j) {
    auto it = grids.find(j.key);
    if (it != grids.end()) {
      j.g = it->second;
      return BHAH_OK;
    }
    bhah_grid* g = nullptr;
    const int rc = bhah_grid_create(&j.d.grid, &g);
    if (rc) return rc;
    grids[j.key] = g;
    j.g = g;
    return BHAH_OK;
  }

  void release(Job& j) {
    if (j.mem) free_slabs[j.key].push_back(j.mem);
    j.mem = nullptr;
  }

  long long running_points() {
    long long n = 0;
    for (long long id : running) n += jobs[id].g->info.n_interior;
    return n;
  }

  // admit queued jobs in arrival order while a slot and memory are free and
  // the running set is below the target size
  int admit() {
    long long pts = running_points();
    for (auto it = queue.begin(); it != queue.end();) {
      if ((int)running.size() >= p.max_jobs) break;
      if (p.target_points > 0 && pts >= p.target_points) break;
      Job& j = jobs[*it];
      std::vector<double*>& fl = free_slabs[j.key];
      double* mem = nullptr;
      if (!fl.empty()) {
        mem = fl.back();
        fl.pop_back();
      } else {
        const double need = slab_bytes(j.g);
        if (held + need > p.budget_bytes) {
          ++it;
          continue;
        }
        if (hipMalloc((void**)&mem, (size_t)need) != hipSuccess) {
          (void)hipGetLastError();
          ++it;
          continue;
        }
        all_slabs.push_back(mem);
        held += need;
        peak_held = std::max(peak_held, held);
      }
      j.mem = mem;
      int rc = bhah_set_initial_data_brill_lindquist(j.g, j.d.n_punct, j.d.masses, &j.d.pos[0][0],
                                                     j.d.lapse_kind, mem, stream);
      if (rc) return rc;
      j.state = BHAH_JOB_RUNNING;
      j.t_admit = now();
      pts += j.g->info.n_interior;
      running.push_back(*it);
      it = queue.erase(it);
    }
    peak_running = std::max(peak_running, (int)running.size());
    return BHAH_OK;
  }
};

extern "C" {

int bhah_server_create(const bhah_server_params* p, void* stream, bhah_server** out) {
  if (!p || !out) return bhah::fail(BHAH_EINVAL, "bhah_server_create: NULL argument");
  if (p->max_jobs < 1 || p->steps_per_tick < 1 || !(p->budget_bytes > 0))
    return bhah::fail(BHAH_EINVAL, "bhah_server_create: max_jobs, steps_per_tick and budget must be positive");
  if (int rc = bhah::check_gauge(&p->gauge, "bhah_server_create")) return rc;
  if (p->integrator != BHAH_RK4 && p->integrator != BHAH_SSPRK3)
    return bhah::fail(BHAH_EINVAL, "bhah_server_create: integrator must be BHAH_RK4 or BHAH_SSPRK3");
  bhah_server* s = new (std::nothrow) bhah_server(*p, (hipStream_t)stream);
  if (!s) return bhah::fail(BHAH_ENOMEM, "bhah_server_create: host allocation failed");
  s->engine.set_graph_steps(p->steps_per_tick);
  s->engine.set_integrator(p->integrator);
  *out = s;
  return BHAH_OK;
}

int bhah_server_submit(bhah_server* s, const bhah_job_desc* job, long long* id) {
  if (!s || !job || !id) return bhah::fail(BHAH_EINVAL, "bhah_server_submit: NULL argument");
  if (job->n_punct < 0 || job->n_punct > 16 || job->nsteps < 0)
    return bhah::fail(BHAH_EINVAL, "bhah_server_submit: 0 <= n_punct <= 16 and nsteps >= 0 required");
  bhah_server::Job j;
  j.d = *job;
  j.key = grid_key(job->grid);
  int rc = s->grid_for(j);
  if (rc) return rc;
  if (bhah_server::slab_bytes(j.g) > s->p.budget_bytes)
    return bhah::fail(BHAH_EINVAL, "bhah_server_submit: one job needs more than the memory budget");
  j.t_submit = s->now();
  const long long k = s->next_id++;
  s->jobs[k] = j;
  s->queue.push_back(k);
  *id = k;
  return BHAH_OK;
}

int bhah_server_tick(bhah_server* s, int* running, int* queued) {
  if (!s) return bhah::fail(BHAH_EINVAL, "bhah_server_tick: NULL server");
  int rc = s->admit();
  if (rc) return rc;
  // jobs asking for zero steps finish at once
  long long k = s->p.steps_per_tick;
  std::vector<bhah::EngineJob> ej;
  for (long long id : s->running) {
    bhah_server::Job& j = s->jobs[id];
    k = std::min(k, j.d.nsteps - j.done);
    ej.push_back(bhah::EngineJob{j.g, j.mem, j.mem + j.g->info.state_doubles, j.g->info.dt});
  }
  if (!s->running.empty() && k > 0) {
    if ((rc = s->engine.set_jobs(ej))) return rc;
    const double ta = s->now();
    if ((rc = s->engine.step((int)k, s->stream))) return rc;
    if ((rc = bhah::check_hip(hipStreamSynchronize(s->stream), "bhah_server_tick"))) return rc;
    const double dtk = s->now() - ta;
    s->busy += dtk;
    s->step_ms.emplace_back(1e3 * dtk / (double)k, (double)(k * (long long)s->running.size()));
    for (long long id : s->running) {
      bhah_server::Job& j = s->jobs[id];
      j.done += k;
      s->point_steps += k * j.g->info.n_interior;
    }
  } else if (!s->running.empty()) {
    if ((rc = bhah::check_hip(hipStreamSynchronize(s->stream), "bhah_server_tick"))) return rc;
  }
  // retire
  const double t = s->now();
  std::vector<long long> still;
  for (long long id : s->running) {
    bhah_server::Job& j = s->jobs[id];
    if (j.done >= j.d.nsteps) {
      j.state = BHAH_JOB_DONE;
      j.t_done = t;
      s->n_done++;
      s->job_s.emplace_back(j.t_done - j.t_submit, 1.0);
      if (!s->p.keep_results) {
        s->release(j);
        j.state = BHAH_JOB_RELEASED;
      }
    } else {
      still.push_back(id);
    }
  }
  s->running.swap(still);
  if (running) *running = (int)s->running.size();
  if (queued) *queued = (int)s->queue.size();
  return BHAH_OK;
}

int bhah_server_job_status(const bhah_server* s, long long id, bhah_job_status* st) {
  if (!s || !st) return bhah::fail(BHAH_EINVAL, "bhah_server_job_status: NULL argument");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return bhah::fail(BHAH_EINVAL, "bhah_server_job_status: unknown job");
  const bhah_server::Job& j = it->second;
  st->state = j.state;
  st->steps_done = j.done;
  st->interior_points = j.g->info.n_interior;
  st->t_submit = j.t_submit;
  st->t_admit = j.t_admit;
  st->t_done = j.t_done;
  return BHAH_OK;
}

int bhah_server_fetch(bhah_server* s, long long id, double* dst) {
  if (!s || !dst) return bhah::fail(BHAH_EINVAL, "bhah_server_fetch: NULL argument");
  if (int rc = bhah::check_aligned("bhah_server_fetch", {dst})) return rc;
  auto it = s->jobs.find(id);
  if (it == s->jobs.end() || it->second.state != BHAH_JOB_DONE)
    return bhah::fail(BHAH_EINVAL, "bhah_server_fetch: job unknown, not finished or already released");
  bhah_server::Job& j = it->second;
  const size_t bytes = sizeof(double) * (size_t)j.g->info.state_doubles;
  int rc = bhah::check_hip(hipMemcpyAsync(dst, j.mem, bytes, hipMemcpyDeviceToDevice, s->stream), "fetch copy");
  if (!rc) rc = bhah::check_hip(hipStreamSynchronize(s->stream), "fetch copy");
  if (rc) return rc;
  s->release(j);
  j.state = BHAH_JOB_RELEASED;
  return BHAH_OK;
}

int bhah_server_get_stats(const bhah_server* s, bhah_server_stats* st) {
  if (!s || !st) return bhah::fail(BHAH_EINVAL, "bhah_server_get_stats: NULL argument");
  st->submitted = s->next_id - 1;
  st->done = s->n_done;
  st->running = (long long)s->running.size();
  st->queued = (long long)s->queue.size();
  st->point_steps = s->point_steps;
  st->busy_seconds = s->busy;
  st->elapsed_seconds = s->now();
  st->step_ms_p50 = weighted_percentile(s->step_ms, 50);
  st->step_ms_p99 = weighted_percentile(s->step_ms, 99);
  st->job_s_p50 = weighted_percentile(s->job_s, 50);
  st->job_s_p99 = weighted_percentile(s->job_s, 99);
  st->held_bytes = s->held;
  st->peak_held_bytes = s->peak_held;
  st->peak_running = s->peak_running;
  return BHAH_OK;
}

void bhah_server_destroy(bhah_server* s) { delete s; }

}  // extern "C"
