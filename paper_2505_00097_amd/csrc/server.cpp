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
    long long launched = 0;  // steps enqueued on the device
    long long done = 0;      // steps known to be complete
    double t_submit = -1, t_admit = -1, t_done = -1;
  };
  // one tick's device work: its events and the steps each job took in it
  struct Tick {
    hipEvent_t start = nullptr, end = nullptr;
    std::vector<std::pair<long long, long long>> ran;  // (job, steps)
    int k = 0;                                          // steps of the graph
    bool live = false;
  };

  bhah_server_params p;
  hipStream_t stream;
  bhah::Engine engine;
  double t0;
  // host time of the reference event: device event times map onto the
  // host clock as t_ref + elapsed(ref, event)
  hipEvent_t ref = nullptr;
  double t_ref = 0.0;
  Tick ticks[2];
  int cur = 0;
  std::map<std::string, bhah_grid*> grids;
  std::map<std::string, std::vector<double*>> free_slabs;
  std::map<double*, double> slab_bytes_of;  // every slab held, with its size
  double held = 0.0, peak_held = 0.0;
  std::unordered_map<long long, Job> jobs;
  std::deque<long long> queue;
  std::vector<long long> running;
  long long in_flight = 0;  // jobs whose last steps are enqueued but not yet complete
  long long next_id = 1;
  long long n_done = 0, n_failed = 0;
  long long point_steps = 0;
  double busy = 0.0;
  int peak_running = 0;
  std::vector<std::pair<double, double>> step_ms;  // (latency, job-steps)
  std::vector<std::pair<double, double>> job_s;    // (latency, 1)

  bhah_server(const bhah_server_params& prm, hipStream_t s)
      : p(prm), stream(s), engine(prm.gauge, prm.tune_cache_path), t0(now_s()) {}
  ~bhah_server() {
    (void)hipStreamSynchronize(stream);
    for (auto& kv : slab_bytes_of) (void)hipFree(kv.first);
    for (auto& kv : grids) bhah_grid_destroy(kv.second);
    for (Tick& t : ticks) {
      if (t.start) (void)hipEventDestroy(t.start);
      if (t.end) (void)hipEventDestroy(t.end);
    }
    if (ref) (void)hipEventDestroy(ref);
  }
  int init() {
    int rc = bhah::check_hip(hipEventCreate(&ref), "hipEventCreate");
    for (Tick& t : ticks) {
      if (!rc) rc = bhah::check_hip(hipEventCreate(&t.start), "hipEventCreate");
      if (!rc) rc = bhah::check_hip(hipEventCreate(&t.end), "hipEventCreate");
    }
    if (!rc) rc = bhah::check_hip(hipEventRecord(ref, stream), "hipEventRecord");
    if (!rc) rc = bhah::check_hip(hipEventSynchronize(ref), "hipEventSynchronize");
    t_ref = now();
    return rc;
  }
  double now() const { return now_s() - t0; }
  double event_time(hipEvent_t e) const {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ref, e) != hipSuccess) return now();
    return t_ref + 1e-3 * (double)ms;
  }
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

  // a released slab goes back to the free list of its grid shape; work
  // already enqueued on the stream may still write it, and whatever reuses
  // it is enqueued after that work
  void release(Job& j) {
    if (j.mem) free_slabs[j.key].push_back(j.mem);
    j.mem = nullptr;
  }

  // free slabs of grid shapes other than `key` until `need` more bytes fit
  // the budget (after the stream has drained: a released slab may still be
  // written by enqueued work)
  int reclaim(const std::string& key, double need) {
    bool synced = false;
    for (auto& kv : free_slabs) {
      if (kv.first == key) continue;
      while (!kv.second.empty() && held + need > p.budget_bytes) {
        if (!synced) {
          if (int rc = bhah::check_hip(hipStreamSynchronize(stream), "bhah_server_tick")) return rc;
          synced = true;
        }
        double* m = kv.second.back();
        kv.second.pop_back();
        held -= slab_bytes_of[m];
        slab_bytes_of.erase(m);
        if (int rc = bhah::check_hip(hipFree(m), "hipFree")) return rc;
      }
    }
    return BHAH_OK;
  }

  long long running_points() {
    long long n = 0;
    for (long long id : running) n += jobs[id].g->info.n_interior;
    return n;
  }

  // admit queued jobs in arrival order while a slot and memory are free and
  // the running set is below the target size; a job whose initial data
  // cannot be set is marked failed and leaves the queue
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
        if (held + need > p.budget_bytes)
          if (int rc = reclaim(j.key, need)) return rc;
        if (held + need > p.budget_bytes) {
          ++it;
          continue;
        }
        if (hipMalloc((void**)&mem, (size_t)need) != hipSuccess) {
          (void)hipGetLastError();
          ++it;
          continue;
        }
        slab_bytes_of[mem] = need;
        held += need;
        peak_held = std::max(peak_held, held);
      }
      j.mem = mem;
      const int rc = bhah_set_initial_data_brill_lindquist(j.g, j.d.n_punct, j.d.masses, &j.d.pos[0][0],
                                                           j.d.lapse_kind, mem, stream);
      if (rc) {
        release(j);
        j.state = BHAH_JOB_FAILED;
        n_failed++;
        it = queue.erase(it);
        if (rc == BHAH_EDEVICE) return rc;
        continue;
      }
      j.state = BHAH_JOB_RUNNING;
      j.t_admit = now();
      pts += j.g->info.n_interior;
      running.push_back(*it);
      it = queue.erase(it);
    }
    peak_running = std::max(peak_running, (int)running.size());
    return BHAH_OK;
  }

  // account for a tick whose device work has completed
  void complete(Tick& t) {
    if (!t.live) return;
    float ms = 0.f;
    if (t.k > 0 && hipEventElapsedTime(&ms, t.start, t.end) == hipSuccess) {
      busy += 1e-3 * (double)ms;
      long long js = 0;
      for (auto& r : t.ran) js += r.second;
      if (js > 0) step_ms.emplace_back((double)ms / (double)t.k, (double)js);
    }
    const double te = event_time(t.end);
    for (auto& r : t.ran) {
      Job& j = jobs[r.first];
      j.done += r.second;
      point_steps += r.second * j.g->info.n_interior;
      if (j.done >= j.d.nsteps) {
        j.state = p.keep_results ? BHAH_JOB_DONE : BHAH_JOB_RELEASED;
        j.t_done = te;
        n_done++;
        in_flight--;
        job_s.emplace_back(j.t_done - j.t_submit, 1.0);
      }
    }
    t.ran.clear();
    t.live = false;
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
  if (int rc = s->init()) {
    delete s;
    return rc;
  }
  s->engine.set_graph_steps(p->steps_per_tick);
  s->engine.set_integrator(p->integrator);
  *out = s;
  return BHAH_OK;
}

int bhah_server_submit(bhah_server* s, const bhah_job_desc* job, long long* id) {
  if (!s || !job || !id) return bhah::fail(BHAH_EINVAL, "bhah_server_submit: NULL argument");
  if (job->n_punct < 0 || job->n_punct > 16 || job->nsteps < 0)
    return bhah::fail(BHAH_EINVAL, "bhah_server_submit: 0 <= n_punct <= 16 and nsteps >= 0 required");
  if (job->lapse_kind != 0 && job->lapse_kind != 1)
    return bhah::fail(BHAH_EINVAL, "bhah_server_submit: lapse_kind must be 0 (psi^-2) or 1 (one)");
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
  // this tick: every running job takes min(steps left, steps_per_tick)
  // steps, all in one graph launch of the largest of those counts
  bhah_server::Tick& t = s->ticks[s->cur];
  long long k = 0;
  std::vector<bhah::EngineJob> ej;
  std::vector<long long> still;
  for (long long id : s->running) {
    bhah_server::Job& j = s->jobs[id];
    const long long n = std::min<long long>(s->p.steps_per_tick, j.d.nsteps - j.launched);
    k = std::max(k, n);
    if (n > 0) {
      bhah::EngineJob e{j.g, j.mem, j.mem + j.g->info.state_doubles, j.g->info.dt};
      e.limit = n;
      ej.push_back(e);
    }
    t.ran.emplace_back(id, n);
    j.launched += n;
    if (j.launched >= j.d.nsteps) {
      // its last steps are enqueued: the slot is free for the next tick
      s->in_flight++;
      if (!s->p.keep_results) s->release(j);
    } else {
      still.push_back(id);
    }
  }
  if ((rc = bhah::check_hip(hipEventRecord(t.start, s->stream), "hipEventRecord"))) return rc;
  if (k > 0) {
    if ((rc = s->engine.set_jobs(ej))) return rc;
    if ((rc = s->engine.step((int)k, s->stream))) return rc;
  }
  if ((rc = bhah::check_hip(hipEventRecord(t.end, s->stream), "hipEventRecord"))) return rc;
  t.k = (int)k;
  t.live = true;
  s->running.swap(still);
  // at most one tick stays in flight: wait for the previous one, whose
  // completion makes its jobs' results final
  s->cur ^= 1;
  bhah_server::Tick& prev = s->ticks[s->cur];
  if (prev.live) {
    if ((rc = bhah::check_hip(hipEventSynchronize(prev.end), "bhah_server_tick"))) return rc;
    s->complete(prev);
  }
  // with nothing running or queued, finish this tick too (drain)
  if (s->running.empty() && s->queue.empty()) {
    if ((rc = bhah::check_hip(hipEventSynchronize(t.end), "bhah_server_tick"))) return rc;
    s->complete(t);
  }
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
  st->running = (long long)s->running.size() + s->in_flight;
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
  st->failed = s->n_failed;
  return BHAH_OK;
}

void bhah_server_destroy(bhah_server* s) { delete s; }

}  // extern "C"
