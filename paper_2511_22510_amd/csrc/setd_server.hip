// setd_server.hip -- continuous-batching job server of the C ABI.
//
// A scheduler thread owns the caller's stream and device arena.  Submitted
// jobs wait in a queue and are admitted, first fit in arrival order, when
// their workspace fits a free block of the arena and a slot is free; a job
// waiting longer than the aging limit stops later jobs from overtaking it.
// Every scheduler tick advances all admitted jobs together: realizations of
// jobs of the same launch class (lattice, field type, precision, dealiasing,
// kind of nonlinearity) form one item table and share one launch per pass,
// each item taking its own number of steps in the tick.  Jobs admitted while
// a tick runs join the next one.  A finished job's observables and final
// state are kept on the host and its arena block is freed at once.
//
// A job's trajectory depends only on its descriptor: every item carries its
// own state, coefficients, seed and step counter, so it is the same alone and
// in any mix (the kernels do the same arithmetic for any batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "setd_launch.hpp"
#include "setd_runtime.hpp"

namespace setd {

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

static double env_double(const char* name, double dflt)
{
    const char* v = std::getenv(name);
    return v ? std::atof(v) : dflt;
}

// First-fit allocator over [0, size) with coalescing of freed blocks.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t n)
    {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t* off)
    {
        n = (n + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t roff = it->first + n;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + 255) / 256 * 256;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum JobState { JOB_QUEUED = 0, JOB_ACTIVE = 1, JOB_DONE = 2 };

struct Job {
    setd_job id = 0;
    setd_desc d{};
    int64_t nsteps = 0, done_steps = 0;
    std::unique_ptr<Plan> plan;
    size_t off = 0, bytes = 0;
    size_t nitems = 0;   // entries of the per-tick item table the job takes
    int state = JOB_QUEUED;
    setd_status status = SETD_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int steps_tick = 0;
    // results kept after the job's arena block is freed
    std::vector<double> obs_sk, obs_width, obs_step;
    std::vector<char> final_state;   // R stored blocks, state precision
    bool have_state = false;
};

}  // namespace setd

using namespace setd;

struct setd_server {
    char* arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t stream = nullptr;
    // launch classes of a tick are independent: each runs on one of these
    // streams, forked from and joined back into `stream` with events, so that
    // small lattices of different classes share the GPU
    static constexpr int NLANE = 4;
    int nlanes = 0;
    hipStream_t lanes[NLANE] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_lane[NLANE] = {};
    Arena alloc;
    // device item tables, one region per launch class of a tick; items_used
    // counts the entries the active jobs take (admission keeps it <= items_cap)
    size_t items_off = 0, items_cap = 0, items_used = 0;
    Item* items_host = nullptr;   // pinned

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<setd_job, std::unique_ptr<Job>> jobs;
    std::deque<setd_job> queue;
    std::vector<setd_job> active;
    setd_job next_id = 1;
    bool stop = false;
    std::thread worker;
    int max_active = 256;
    double aging_s = 1.0;
    double tick_target_s = 0.005;
    size_t keep_budget = (size_t)2 << 30;   // host bytes of retained final states
    size_t kept_bytes = 0;
    std::deque<setd_job> kept_order;
    double est_step_s = 0.0;              // measured wall time of one batched step
    // 2D real-field classes of different lattice sizes share one launch per
    // pass (SETD_SERVER_MULTI=0 keeps a launch per class)
    bool multi = true;
    // counters: ticks that ran steps, pass launches queued, shared ones among them
    double n_ticks = 0, n_launches = 0, n_shared = 0;

    void run();
    void admit_locked(std::vector<Job*>& admitted);
    // a job leaves the active set: its arena block and item entries are freed
    void retire_locked(Job* j, setd_status st);
    setd_status tick(std::vector<Job*>& act, int* steps_taken);
    void finish(Job* j);
    void retain(Job* j);
};

void setd_server::admit_locked(std::vector<Job*>& admitted)
{
    const double t = now_s();
    bool blocked = false;
    for (auto qi = queue.begin(); qi != queue.end();) {
        if ((int)active.size() >= max_active) break;
        Job* j = jobs[*qi].get();
        size_t off = 0;
        if (!blocked && items_used + j->nitems <= items_cap && alloc.alloc(j->bytes, &off)) {
            j->off = off;
            j->state = JOB_ACTIVE;
            j->t_admit = t;
            items_used += j->nitems;
            active.push_back(j->id);
            admitted.push_back(j);
            qi = queue.erase(qi);
            continue;
        }
        // a job that has waited beyond the aging limit is not overtaken
        if (t - j->t_submit > aging_s) blocked = true;
        if (blocked) break;
        ++qi;
    }
}

void setd_server::retire_locked(Job* j, setd_status st)
{
    j->status = st;
    j->state = JOB_DONE;
    j->t_done = now_s();
    alloc.release(j->off, j->bytes);
    items_used -= j->nitems;
    active.erase(std::remove(active.begin(), active.end(), j->id), active.end());
}

void setd_server::retain(Job* j)
{
    const size_t b = j->final_state.size();
    kept_bytes += b;
    kept_order.push_back(j->id);
    while (kept_bytes > keep_budget && !kept_order.empty()) {
        auto it = jobs.find(kept_order.front());
        kept_order.pop_front();
        if (it == jobs.end() || !it->second->have_state) continue;
        kept_bytes -= it->second->final_state.size();
        std::vector<char>().swap(it->second->final_state);
        it->second->have_state = false;
    }
}

// Observables and final state of a job whose last step has run; frees its
// arena block.  Runs on the scheduler thread.
void setd_server::finish(Job* j)
{
    Plan& p = *j->plan;
    int flag = 0;
    std::vector<double> buf(3 * (size_t)p.nbins + 8);
    size_t len = 0;
    // a plan keeping the SETD2 carry recovers phi before it is read
    const setd_status rec = p.ensure_phi();
    setd_status st = SETD_OK;
    if (p.iso && p.observe(SETD_OBS_SK, buf.data(), buf.size(), &len) != SETD_E_DEVICE)
        j->obs_sk.assign(buf.begin(), buf.begin() + len);
    if (p.observe(SETD_OBS_WIDTH, buf.data(), buf.size(), &len) != SETD_E_DEVICE)
        j->obs_width.assign(buf.begin(), buf.begin() + len);
    st = p.observe(SETD_OBS_STEP, buf.data(), buf.size(), &len);
    if (st == SETD_OK || st == SETD_E_NONFINITE) j->obs_step.assign(buf.begin(), buf.begin() + len);
    if (p.nonfinite_any(&flag) != SETD_OK || rec != SETD_OK) st = SETD_E_DEVICE;
    std::vector<char> raw((size_t)p.R * p.Sb);
    if (hipMemcpyAsync(raw.data(), p.ws + p.lay.phi, raw.size(), hipMemcpyDeviceToHost, stream) == hipSuccess &&
        hipStreamSynchronize(stream) == hipSuccess) {
        j->final_state.swap(raw);
        j->have_state = true;
    }
    std::lock_guard<std::mutex> lk(mu);
    retire_locked(j, (st == SETD_E_DEVICE) ? SETD_E_DEVICE : (flag ? SETD_E_NONFINITE : SETD_OK));
    if (j->have_state) retain(j);
}

// One scheduler tick: every active job advances min(remaining, chunk) steps.
setd_status setd_server::tick(std::vector<Job*>& act, int* steps_taken)
{
    // steps per tick: about tick_target_s of GPU time, at least 1
    int chunk = 16;
    if (est_step_s > 0) chunk = (int)std::max(1.0, std::min(1024.0, tick_target_s / est_step_s));
    std::map<std::string, std::vector<Job*>> classes;
    int maxk = 0;
    for (Job* j : act) {
        j->steps_tick = (int)std::min<int64_t>(chunk, j->nsteps - j->done_steps);
        maxk = std::max(maxk, j->steps_tick);
        classes[class_key(*j->plan)].push_back(j);
    }
    // item tables, one contiguous run per class.  A real 1D line pairs
    // realizations 2l and 2l + 1 in one transform, whose rounding couples
    // them: a job with an odd count gets a partner that never steps (a copy
    // of its last item with no steps), so that every job's realizations pair
    // as in a solo run.
    auto padded = [](const Job* j) { return j->nitems > (size_t)j->plan->R; };
    size_t nitems = 0;
    for (auto& c : classes)
        for (Job* j : c.second) nitems += j->nitems;
    // admission keeps the active jobs' entries within the table
    if (nitems > items_cap) return fail(SETD_E_NOMEM, "item table overflow");
    size_t pos = 0;
    struct Launch { Plan* rep; size_t first; int n; };
    std::vector<Launch> launches;
    for (auto& c : classes) {
        const size_t first = pos;
        for (Job* j : c.second) {
            for (int r = 0; r < j->plan->R; r++) {
                Item it = j->plan->items[r];
                it.steps = j->steps_tick;
                items_host[pos++] = it;
            }
            if (padded(j)) {
                Item it = j->plan->items[j->plan->R - 1];
                it.steps = 0;
                items_host[pos++] = it;
            }
        }
        launches.push_back({c.second.front()->plan.get(), first, (int)(pos - first)});
    }
    Item* items_dev = reinterpret_cast<Item*>(arena + items_off);
    SETD_HIP(hipMemcpyAsync(items_dev, items_host, nitems * sizeof(Item), hipMemcpyHostToDevice, stream));
    // launch units: the classes that can share launches (one per lattice
    // size, multi2d_ok) form one unit when there are two or more of them;
    // every other class is a unit of its own (-1 marks the shared unit)
    MultiClass mc[4] = {};
    int nshare = 0;
    if (multi)
        for (const Launch& L : launches)
            if (multi2d_ok(L.rep->g, L.rep->lean, L.rep->d.nl)) nshare++;
    std::vector<int> units;
    if (nshare >= 2) units.push_back(-1);
    for (size_t c = 0; c < launches.size(); c++) {
        const Launch& L = launches[c];
        if (nshare >= 2 && multi2d_ok(L.rep->g, L.rep->lean, L.rep->d.nl))
            mc[multi2d_slot(L.rep->g.n[0])] = MultiClass{L.rep->g, items_dev + L.first, L.n};
        else
            units.push_back((int)c);
    }
    const double t0 = now_s();
    const int nl = std::min<int>(nlanes, (int)units.size());
    if (nl >= 2) {
        SETD_HIP(hipEventRecord(ev_fork, stream));
        for (int i = 0; i < nl; i++) SETD_HIP(hipStreamWaitEvent(lanes[i], ev_fork, 0));
    }
    setd_status lst = SETD_OK;
    double q_launches = 0, q_shared = 0;
    for (int sub = 0; sub < maxk && lst == SETD_OK; sub++) {
        for (size_t u = 0; u < units.size() && lst == SETD_OK; u++) {
            const hipStream_t ls = nl >= 2 ? lanes[u % nl] : stream;
            if (units[u] < 0) {
                for (int pass = 0; pass < 2 && lst == SETD_OK; pass++) {
                    const hipError_t e = launch_multi2d<float>(mc, pass, sub, ls);
                    if (e != hipSuccess) lst = fail(SETD_E_DEVICE, "shared launch failed: %s", hipGetErrorString(e));
                }
                q_launches += 2;
                q_shared += 2;
            } else {
                const Launch& L = launches[units[u]];
                lst = L.rep->launch_step(items_dev + L.first, L.n, sub, ls);
                q_launches += L.rep->passes_per_step();
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        n_launches += q_launches;
        n_shared += q_shared;
        if (maxk > 0) n_ticks += 1;
    }
    if (nl >= 2) {
        // join even after a failed launch
        for (int i = 0; i < nl; i++) {
            SETD_HIP(hipEventRecord(ev_lane[i], lanes[i]));
            SETD_HIP(hipStreamWaitEvent(stream, ev_lane[i], 0));
        }
    }
    if (lst != SETD_OK) return lst;
    SETD_HIP(hipStreamSynchronize(stream));
    const double dt = now_s() - t0;
    if (maxk > 0) {
        const double per = dt / maxk;
        est_step_s = (est_step_s > 0) ? 0.7 * est_step_s + 0.3 * per : per;
    }
    for (Job* j : act) {
        j->done_steps += j->steps_tick;
        if (j->steps_tick > 0 && j->plan->lean) j->plan->phi_valid = false;
    }
    *steps_taken = maxk;
    return SETD_OK;
}

void setd_server::run()
{
    for (;;) {
        std::vector<Job*> admitted, act;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop) return;
            admit_locked(admitted);
            for (setd_job id : active) act.push_back(jobs[id].get());
        }
        // bind the new jobs: tables, tuned variants, initial condition
        for (Job* j : admitted) {
            setd_status st = j->plan->bind(arena + j->off, j->bytes, stream);
            if (st != SETD_OK) {
                std::lock_guard<std::mutex> lk(mu);
                retire_locked(j, st);
                act.erase(std::remove(act.begin(), act.end(), j), act.end());
            }
        }
        if (!act.empty()) {
            int taken = 0;
            setd_status st = tick(act, &taken);
            if (st != SETD_OK) {
                // a device failure ends every job of the tick
                std::lock_guard<std::mutex> lk(mu);
                for (Job* j : act) retire_locked(j, st);
            } else {
                for (Job* j : act)
                    if (j->done_steps >= j->nsteps) finish(j);
            }
        }
        cv_done.notify_all();
    }
}

// ====================================================================== C ABI
extern "C" {

double setd_clock(void) { return now_s(); }

setd_status setd_server_create(void* dev_arena, size_t bytes, void* hip_stream, setd_server** out)
{
    if (!dev_arena || !out) return fail(SETD_E_INVAL, "null argument");
    if (((uintptr_t)dev_arena) % 256 != 0) return fail(SETD_E_INVAL, "arena must be 256-byte aligned");
    // entries of the per-tick item table (SETD_SERVER_ITEMS, default 16384)
    const size_t items_cap = (size_t)std::max(2.0, std::min(1048576.0, env_double("SETD_SERVER_ITEMS", 16384)));
    const size_t table = (items_cap * sizeof(Item) + 255) / 256 * 256;
    if (bytes < table + (1u << 20)) return fail(SETD_E_NOMEM, "arena too small");
    setd_server* s = new (std::nothrow) setd_server();
    if (!s) return fail(SETD_E_NOMEM, "host allocation failed");
    s->arena = (char*)dev_arena;
    s->arena_bytes = bytes;
    s->stream = (hipStream_t)hip_stream;
    s->items_off = 0;
    s->items_cap = items_cap;
    if (hipHostMalloc((void**)&s->items_host, items_cap * sizeof(Item), hipHostMallocDefault) != hipSuccess) {
        delete s;
        return fail(SETD_E_DEVICE, "pinned host allocation failed");
    }
    // jobs live above the item table
    s->alloc.init(bytes - table);
    s->items_off = bytes - table;
    s->max_active = (int)env_double("SETD_SERVER_SLOTS", 256);
    s->aging_s = env_double("SETD_SERVER_AGING", 1.0);
    s->tick_target_s = env_double("SETD_SERVER_TICK", 0.005);
    s->keep_budget = (size_t)env_double("SETD_SERVER_KEEP_BYTES", (double)((size_t)2 << 30));
    s->multi = env_double("SETD_SERVER_MULTI", 1) != 0;
    // SETD_SERVER_LANES (0..4, default 4) streams for the launch classes of a tick
    const int want = std::max(0, std::min(setd_server::NLANE, (int)env_double("SETD_SERVER_LANES", 4)));
    if (want >= 2 && hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) == hipSuccess) {
        for (int i = 0; i < want; i++) {
            if (hipStreamCreateWithFlags(&s->lanes[i], hipStreamNonBlocking) != hipSuccess) break;
            if (hipEventCreateWithFlags(&s->ev_lane[i], hipEventDisableTiming) != hipSuccess) {
                (void)hipStreamDestroy(s->lanes[i]);
                s->lanes[i] = nullptr;
                break;
            }
            s->nlanes = i + 1;
        }
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return SETD_OK;
}

setd_status setd_submit(setd_server* s, const setd_desc* desc, int64_t nsteps, setd_job* out)
{
    if (!s || !desc || !out) return fail(SETD_E_INVAL, "null argument");
    if (nsteps < 0 || nsteps >= ((int64_t)1 << 32)) return fail(SETD_E_INVAL, "step count out of range");
    std::unique_ptr<Job> j(new (std::nothrow) Job());
    if (!j) return fail(SETD_E_NOMEM, "host allocation failed");
    j->plan.reset(new (std::nothrow) Plan());
    if (!j->plan) return fail(SETD_E_NOMEM, "host allocation failed");
    setd_status st = j->plan->init(*desc);
    // the scheduler batches jobs into its own launches on the server stream
    j->plan->split_ok = false;
    if (st != SETD_OK) return st;
    j->d = *desc;
    j->nsteps = nsteps;
    j->bytes = j->plan->lay.total;
    // a real 1D line with an odd realization count takes one padding entry
    const Plan& jp = *j->plan;
    j->nitems = (size_t)jp.R + ((jp.g.ndim == 1 && !jp.g.cplx && (jp.R % 2) == 1) ? 1 : 0);
    if (j->nitems > s->items_cap)
        return fail(SETD_E_INVAL, "job takes %zu item entries, the server's table holds %zu", j->nitems, s->items_cap);
    if (j->bytes > s->alloc.size) return fail(SETD_E_NOMEM, "job needs %zu bytes, arena has %zu", j->bytes, s->alloc.size);
    std::lock_guard<std::mutex> lk(s->mu);
    j->id = s->next_id++;
    j->t_submit = now_s();
    *out = j->id;
    s->queue.push_back(j->id);
    s->jobs[j->id] = std::move(j);
    s->cv_work.notify_one();
    return SETD_OK;
}

setd_status setd_poll(setd_server* s, setd_job job, int* done, setd_status* job_status)
{
    if (!s || !done || !job_status) return fail(SETD_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(SETD_E_INVAL, "unknown job %lld", (long long)job);
    *done = it->second->state == JOB_DONE;
    *job_status = *done ? it->second->status : SETD_E_BUSY;
    return SETD_OK;
}

setd_status setd_server_drain(setd_server* s)
{
    if (!s) return fail(SETD_E_INVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->queue.empty() && s->active.empty(); });
    return SETD_OK;
}

setd_status setd_job_observe(setd_server* s, setd_job job, int kind, double* out, size_t cap, size_t* len)
{
    if (!s || !out || !len) return fail(SETD_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(SETD_E_INVAL, "unknown job %lld", (long long)job);
    Job* j = it->second.get();
    if (j->state != JOB_DONE) return fail(SETD_E_BUSY, "job still running");
    const std::vector<double>* v = nullptr;
    if (kind == SETD_OBS_SK) v = &j->obs_sk;
    else if (kind == SETD_OBS_WIDTH) v = &j->obs_width;
    else if (kind == SETD_OBS_STEP) v = &j->obs_step;
    else return fail(SETD_E_INVAL, "finished jobs keep SK, WIDTH and STEP");
    if (v->empty()) return fail(SETD_E_INVAL, "observable not available for this job");
    if (cap < v->size()) return fail(SETD_E_INVAL, "output needs %zu doubles", v->size());
    std::copy(v->begin(), v->end(), out);
    *len = v->size();
    return j->status == SETD_E_NONFINITE ? fail(SETD_E_NONFINITE, "the job produced a non-finite value") : SETD_OK;
}

setd_status setd_job_get_field(setd_server* s, setd_job job, int realization, double* host_out, size_t cap)
{
    if (!s || !host_out) return fail(SETD_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(SETD_E_INVAL, "unknown job %lld", (long long)job);
    Job* j = it->second.get();
    if (j->state != JOB_DONE) return fail(SETD_E_BUSY, "job still running");
    if (!j->have_state) return fail(SETD_E_STATE, "final state not retained (host budget)");
    const Plan& p = *j->plan;
    if (realization < 0 || realization >= p.R) return fail(SETD_E_INVAL, "realization out of range");
    if (cap < 2 * p.nspec) return fail(SETD_E_INVAL, "output needs %zu doubles", 2 * p.nspec);
    p.scatter(j->final_state.data() + (size_t)realization * p.Sb, host_out);
    return SETD_OK;
}

setd_status setd_job_times(setd_server* s, setd_job job, double* out4)
{
    if (!s || !out4) return fail(SETD_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(SETD_E_INVAL, "unknown job %lld", (long long)job);
    const Job* j = it->second.get();
    out4[0] = j->t_submit;
    out4[1] = j->t_admit;
    out4[2] = j->t_done;
    out4[3] = (double)j->done_steps;
    return SETD_OK;
}

setd_status setd_server_stats(setd_server* s, double* out, size_t cap, size_t* len)
{
    if (!s || !out || !len) return fail(SETD_E_INVAL, "null argument");
    if (cap < 3) return fail(SETD_E_INVAL, "output needs 3 doubles");
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->n_ticks;
    out[1] = s->n_launches;
    out[2] = s->n_shared;
    *len = 3;
    return SETD_OK;
}

setd_status setd_server_destroy(setd_server* s)
{
    if (!s) return SETD_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (int i = 0; i < s->nlanes; i++) {
        (void)hipStreamSynchronize(s->lanes[i]);
        (void)hipStreamDestroy(s->lanes[i]);
        (void)hipEventDestroy(s->ev_lane[i]);
    }
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->items_host) (void)hipHostFree(s->items_host);
    delete s;
    return SETD_OK;
}

}  // extern "C"
