// Continuous-batching server for independent HEOM propagations on one GPU.
//
// Requests (a problem, its initial states and step count) are admitted by
// memory footprint into a caller-owned device arena.  Every admitted request
// joins the active set at an RK4-step boundary; each macro-step then advances
// every active propagation by one RK4 step with batched launches: per stage,
// one sigma_0 launch and one bulk launch per kernel variant (precision,
// FMA/MFMA path) whose grid covers the ADO tiles of all active jobs.  The
// arithmetic of a job does not depend on the batch it runs in (fixed
// tile -> ADO mapping, no cross-job reductions), so a result is the same alone
// and in the mix.  Finished requests leave at a step boundary; their records
// are copied to pinned host memory and their arena ranges are freed once the
// copy has completed on the stream.
//
// Two kinds of request leave the batched launches.  A large run gets
// launches of its own on a persistent kernel (its ADOs fill the device):
// FP32 Hermitian runs with 10 <= N <= 64 on the matrix-core one, runs with
// N <= 16 and at least 32768 ADOs on the FMA one.  An eligible dipole request
// (ground state uncoupled, initial states in the (e, g) column, at most three
// directions) runs in the coherence-block form of heom_propagate_block: its
// ADOs keep only their (e, g) column, the three directions side by side
// (section "Linear absorption spectra"), 3N instead of 3 (N+1)^2 elements.
// Both choices depend on the request alone, so results stay the same alone
// and in the mix.
//
// Independent propagations (disorder realisations, dipole directions) are the
// parallelism the paper runs side by side for rotational averages and
// polarisation sequences (section "Distributed memory HEOM implementation").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "heom.h"
#include "heom_internal.h"

namespace {

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr int kMaxRuns = 8;
constexpr size_t kPinnedPool = size_t(256) << 20;
// Runs at least this large get launches of their own (matrix-core and FMA
// persistent kernels; the second matches the FMA kernel's own threshold).
constexpr int64_t kSoloMinAdos = 2048, kSoloSmallMinAdos = 32768;

// First-fit allocator of 256-byte-aligned ranges of [0, size).
class RangeAllocator {
public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align256(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(std::max<size_t>(bytes, 1));
        auto it = free_.emplace(off, bytes).first;
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

private:
    std::map<size_t, size_t> free_;
};

struct Req {
    uint64_t ticket = 0;
    std::vector<double> h_re, h_im, rho0, mu;
    std::vector<heom_bath> baths;
    heom_problem prob{};
    int n_runs = 1, record_every = 1, kind = 0, ground = 0, hermitian = 0;
    int64_t n_steps = 0, n_rec = 0;
    int rd = 0;
    double dt = 0.0;
    heom_info info{};
    size_t state_bytes = 0, work_bytes = 0, footprint = 0, pinned_bytes = 0;
    // runtime
    enum Phase { QUEUED, ACTIVE, DRAINING, DONE } phase = QUEUED;
    heom_hierarchy* h = nullptr;
    size_t arena_off = 0, pinned_off = 0;
    bool has_arena = false, has_pinned = false;
    std::vector<heom::Job> jobs;
    int64_t steps_done = 0;
    hipEvent_t done_ev = nullptr;
    bool cancel = false;
    heom_status status = HEOM_PENDING;
    std::vector<double> records;
    double t_submit = 0.0, t_admit = 0.0, t_finish = 0.0;
    // coherence-block form: the excited-state problem (ground energy 0),
    // observables [3][bN], start column [bN][3] complex, and the device block
    // state, its three stage copies, records [n_rec][6] and status word
    bool block = false;
    int bN = 0;
    std::vector<double> bh_re, bh_im, bobs, bstart;
    std::vector<heom_bath> bbaths;
    heom_problem bprob{};
    heom_info binfo{};
    size_t bstate_bytes = 0, bwork_bytes = 0;
    void* barr[4] = {nullptr, nullptr, nullptr, nullptr};
    double* brec = nullptr;
    double* bobs_dev = nullptr;
    int32_t* bstatus = nullptr;
    int64_t* bstep = nullptr;
    // pinned layout of a block request: start column | obs | records | status
    size_t bpin_obs() const { return align256((size_t)bN * 3 * 16); }
    size_t bpin_rec() const { return bpin_obs() + align256((size_t)3 * bN * 8); }
    size_t bpin_status() const { return bpin_rec() + align256((size_t)n_rec * 6 * 8); }
};

// Device bytes of the job tables at the start of the arena: full-form jobs
// (up to kMaxRuns per request), then one coherence-block job per request.
size_t job_table_bytes(size_t jobs_cap, int max_active) {
    return align256(jobs_cap * sizeof(heom::Job)) + align256((size_t)max_active * sizeof(heom::BlockJob));
}

// A full-form job with launches of its own: FP32 Hermitian runs with
// 10 <= N <= 64 and at least kSoloMinAdos ADOs (the persistent matrix-core
// kernel), and runs with N <= 16 and at least kSoloSmallMinAdos ADOs in
// either precision (the persistent FMA kernel).
bool solo_job(int precision, const heom::Job& j) {
    if (precision == HEOM_FP32_MIXED && j.herm && j.t.N >= 10 && j.t.N <= 64 &&
        j.t.h_complex == 0)
        return j.t.n_ado >= kSoloMinAdos;
    return j.t.N <= 16 && j.t.n_ado >= kSoloSmallMinAdos;
}

struct Group {
    int precision = 0, nb = 0, herm = 0;
    bool solo = false;  // one job, launched on its own
    int job_off = 0, n_jobs = 0, tiles = 0;
    heom::Job sizing{};
};

}  // namespace

struct heom_server {
    char* arena = nullptr;
    size_t arena_bytes = 0;
    int max_active = 1;
    int device = 0;
    hipStream_t stream = nullptr;
    RangeAllocator arena_alloc, pinned_alloc;
    char* pinned = nullptr;
    heom::Job* jobs_dev = nullptr;    // in the arena
    heom::Job* jobs_stage = nullptr;  // pinned staging for the job table
    size_t jobs_cap = 0;
    heom::BlockJob* bjobs_dev = nullptr;    // after the job table
    heom::BlockJob* bjobs_stage = nullptr;  // after its staging
    int n_bjobs = 0;
    int64_t btotal = 0;  // elements of one batched block stage
    hipEvent_t stage_ev = nullptr;
    hipEvent_t step_ev[2] = {nullptr, nullptr};
    int64_t macro = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> pending;
    std::map<uint64_t, std::unique_ptr<Req>> all;
    std::vector<Req*> active, draining;
    uint64_t next_ticket = 1;
    bool stop = false;
    heom_status fatal = HEOM_OK;
    std::string fatal_msg;
    std::vector<Group> groups;
    bool dirty = false;
    std::thread thr;
    std::FILE* log = nullptr;  // per-request JSON lines (heom_server_set_log)

    void run();
    void admit();
    bool setup(Req* r);
    void start_drain(Req* r);
    void finish_draining();
    void finish(Req* r, heom_status st);  // caller holds mu
    void release_resources(Req* r);
    bool rebuild();
    bool launch_macro_step();
    void fail_all(const char* what, hipError_t e);         // takes mu
    void fail_all_locked(const char* what, hipError_t e);  // caller holds mu
};

namespace {

heom_status srv_fail(heom_status s, const std::string& msg) {
    heom::set_last_error(msg);
    return s;
}

}  // namespace

void heom_server::finish(Req* r, heom_status st) {
    r->status = st;
    r->phase = Req::DONE;
    r->t_finish = heom::monotonic_seconds();
    if (log) {
        const bool admitted = r->t_admit > 0.0;
        const double t_admit = admitted ? r->t_admit : r->t_finish;
        std::fprintf(log,
                     "{\"ticket\": %llu, \"status\": %d, \"form\": \"%s\", \"runs\": %d, "
                     "\"n_states\": %d, \"n_ado\": %lld, \"n_steps\": %lld, \"queue_ms\": %.3f, "
                     "\"service_ms\": %.3f, \"latency_ms\": %.3f, \"ado_updates\": %lld}\n",
                     (unsigned long long)r->ticket, (int)st, r->block ? "block" : "full", r->n_runs,
                     r->info.n_states, (long long)r->info.n_ado, (long long)r->n_steps,
                     1e3 * (t_admit - r->t_submit), 1e3 * (r->t_finish - t_admit),
                     1e3 * (r->t_finish - r->t_submit),
                     (long long)(r->info.n_ado * r->n_steps * r->n_runs));
        std::fflush(log);
    }
    cv_done.notify_all();
}

void heom_server::release_resources(Req* r) {
    if (r->h) {
        heom_destroy(r->h);
        r->h = nullptr;
    }
    if (r->has_arena) arena_alloc.release(r->arena_off, r->footprint);
    if (r->has_pinned) pinned_alloc.release(r->pinned_off, r->pinned_bytes);
    r->has_arena = r->has_pinned = false;
    if (r->done_ev) {
        (void)hipEventDestroy(r->done_ev);
        r->done_ev = nullptr;
    }
}

void heom_server::fail_all(const char* what, hipError_t e) {
    std::lock_guard<std::mutex> lk(mu);
    fail_all_locked(what, e);
}

void heom_server::fail_all_locked(const char* what, hipError_t e) {
    fatal = HEOM_E_DEVICE;
    fatal_msg = std::string(what) + ": " + hipGetErrorString(e);
    // Work already enqueued (kernels, record copies) may still touch the
    // requests' ranges: let the stream drain before they are freed and the
    // results published (the error itself may make this return early).
    (void)hipStreamSynchronize(stream);
    for (Req* r : active) {
        release_resources(r);
        finish(r, HEOM_E_DEVICE);
    }
    for (Req* r : draining) {
        release_resources(r);
        finish(r, HEOM_E_DEVICE);
    }
    for (Req* r : pending) finish(r, HEOM_E_DEVICE);
    active.clear();
    draining.clear();
    pending.clear();
    stop = true;
}

// Device and pinned layout of one request (offsets from its ranges):
//   full form   arena: tables | per run: sigma0, rest, workspace
//               pinned: per run: rho0, control block, records, status
//   block form  arena: tables | state | work | observed vectors
//               pinned: start column | observed vectors | records | status
bool heom_server::setup(Req* r) {
    char* base = arena + r->arena_off;
    char* pin = pinned + r->pinned_off;
    hipError_t e;
    if (r->block) {
        // arena: tables | block state | status, three stage copies, records
        heom_status s = heom_build_hierarchy(&r->bprob, base, r->binfo.tables_bytes, stream, &r->h);
        if (s != HEOM_OK) {
            std::lock_guard<std::mutex> lk(mu);
            finish(r, s);
            return false;
        }
        // arena: tables | state | work (status, step counter; three stage
        // copies; records) | observed vectors
        char* st = base + align256(r->binfo.tables_bytes);
        char* w = st + r->bstate_bytes;
        const size_t copy = align256((size_t)r->binfo.n_ado * r->bN * 3 * 16);
        r->barr[0] = st;
        for (int k = 1; k < 4; ++k) r->barr[k] = w + 256 + (size_t)(k - 1) * copy;
        r->bstatus = reinterpret_cast<int32_t*>(w);
        r->bstep = reinterpret_cast<int64_t*>(w + 8);
        r->brec = reinterpret_cast<double*>(w + 256 + 3 * copy);
        r->bobs_dev = reinterpret_cast<double*>(w + r->bwork_bytes);
        const size_t col = (size_t)r->bN * 3 * 16, ob = (size_t)3 * r->bN * 8;
        std::memcpy(pin, r->bstart.data(), col);
        std::memcpy(pin + r->bpin_obs(), r->bobs.data(), ob);
        if ((e = hipMemsetAsync(st, 0, r->bstate_bytes, stream)) ||
            (e = hipMemsetAsync(w, 0, 256, stream)) ||
            (e = hipMemcpyAsync(st, pin, col, hipMemcpyHostToDevice, stream)) ||
            (e = hipMemcpyAsync(r->bobs_dev, pin + r->bpin_obs(), ob, hipMemcpyHostToDevice, stream)) ||
            (e = heom::launch_block_record(st, r->bobs.data(), r->bN, r->brec, r->bstatus, stream))) {
            fail_all("request setup", e);
            return false;
        }
        return true;
    }
    heom_status s = heom_build_hierarchy(&r->prob, base, r->info.tables_bytes, stream, &r->h);
    if (s != HEOM_OK) {
        std::lock_guard<std::mutex> lk(mu);
        finish(r, s);
        return false;
    }
    const int N = r->info.n_states;
    const size_t NN = (size_t)N * N;
    size_t off = align256(r->info.tables_bytes);
    size_t poff = 0;
    r->jobs.clear();
    for (int k = 0; k < r->n_runs; ++k) {
        heom_state st;
        st.sigma0 = base + off;
        off += align256(r->info.sigma0_bytes);
        st.rest = base + off;
        off += align256(std::max<size_t>(r->info.rest_bytes, 1));
        char* work = base + off;
        off += r->work_bytes;
        heom::Job j = heom::bind_workspace(r->h, st, work, r->dt, r->n_steps, r->record_every,
                                           r->kind, r->ground, r->hermitian);
        // initial state: rho0 for sigma_0, zero elsewhere
        char* prho = pin + poff;
        poff += align256(NN * 16);
        std::memcpy(prho, r->rho0.data() + 2 * NN * k, NN * 16);
        char* pctl = pin + poff;
        poff += align256(heom::control_bytes(N));
        std::memset(pctl, 0, heom::control_bytes(N));
        if (r->kind == HEOM_OBS_DIPOLE) std::memcpy(pctl + 1024, r->mu.data() + (size_t)N * k, N * 8);
        poff += align256((size_t)r->n_rec * r->rd * 8) + 256;  // records + status (drain)
        if ((e = hipMemcpyAsync(st.sigma0, prho, NN * 16, hipMemcpyHostToDevice, stream)) ||
            (r->info.rest_bytes &&
             (e = hipMemsetAsync(st.rest, 0, r->info.rest_bytes, stream))) ||
            (e = hipMemcpyAsync(work, pctl, heom::control_bytes(N), hipMemcpyHostToDevice, stream))) {
            fail_all("request setup", e);
            return false;
        }
        r->jobs.push_back(j);
    }
    return true;
}

void heom_server::admit() {
    std::unique_lock<std::mutex> lk(mu);
    while (!pending.empty() && (int)(active.size() + draining.size()) < max_active) {
        Req* r = pending.front();
        if (r->cancel) {
            pending.pop_front();
            finish(r, HEOM_E_CANCELLED);
            continue;
        }
        size_t aoff = 0, poff = 0;
        if (!arena_alloc.alloc(r->footprint, &aoff)) break;
        if (!pinned_alloc.alloc(r->pinned_bytes, &poff)) {
            arena_alloc.release(aoff, r->footprint);
            break;
        }
        pending.pop_front();
        r->arena_off = aoff;
        r->pinned_off = poff;
        r->has_arena = r->has_pinned = true;
        lk.unlock();
        const bool ok = setup(r);
        lk.lock();
        if (!ok) {
            release_resources(r);
            if (r->phase != Req::DONE) finish(r, fatal != HEOM_OK ? fatal : HEOM_E_DEVICE);
            if (stop) return;
            continue;
        }
        r->phase = Req::ACTIVE;
        r->t_admit = heom::monotonic_seconds();
        r->steps_done = 0;
        active.push_back(r);
        dirty = true;
    }
}

bool heom_server::rebuild() {
    groups.clear();
    // key: precision, MFMA blocks, Hermitian path, and -1 for batched jobs
    // or the index of a job launched on its own
    std::map<std::tuple<int, int, int, int>, std::vector<const heom::Job*>> by_key;
    int n_solo = 0;
    for (Req* r : active) {
        if (r->block) continue;
        const int prec = heom::hierarchy_precision(r->h);
        for (const heom::Job& j : r->jobs) {
            const int nb = heom::bulk_mfma_blocks(j.t.N, j.t.h_complex != 0, prec);
            const int solo = solo_job(prec, j) ? n_solo++ : -1;
            by_key[std::make_tuple(prec, nb, nb ? j.herm : 0, solo)].push_back(&j);
        }
    }
    size_t n = 0;
    for (auto& kv : by_key) n += kv.second.size();
    if (n > jobs_cap) {
        fail_all("job table overflow", hipErrorInvalidValue);
        return false;
    }
    if (stage_ev) (void)hipEventSynchronize(stage_ev);  // staging buffer free again
    n_bjobs = 0;
    btotal = 0;
    for (Req* r : active) {
        if (!r->block) continue;
        heom::BlockJob& b = bjobs_stage[n_bjobs++];
        b = heom::BlockJob{};
        b.t = heom::hierarchy_tables(r->h);
        for (int k = 0; k < 4; ++k) b.y[k] = r->barr[k];
        b.dt = r->dt;
        b.elem_begin = btotal;
        b.obs = r->bobs_dev;
        b.rec = r->brec;
        b.status = r->bstatus;
        b.step = r->bstep;
        b.record_every = r->record_every;
        btotal += (int64_t)r->binfo.n_ado * 3 * r->bN;
    }
    int off = 0;
    for (auto& kv : by_key) {
        Group g;
        g.precision = std::get<0>(kv.first);
        g.nb = std::get<1>(kv.first);
        g.herm = std::get<2>(kv.first);
        g.solo = std::get<3>(kv.first) >= 0;
        g.job_off = off;
        g.n_jobs = (int)kv.second.size();
        g.sizing = *kv.second.front();
        int maxN = 0, maxW = 0, maxD = 0, tiles = 0, any_hc = 0;
        size_t fma_bytes = 0;
        for (const heom::Job* j : kv.second) {
            any_hc |= j->t.h_complex != 0;
            if (g.nb == 0)
                fma_bytes = std::max(fma_bytes, heom::fma_lds(j->t.N, j->t.W, j->t.D, j->ados_per_tile,
                                                              g.precision == HEOM_FP64 ? 8 : 4).total);
            heom::Job c = *j;
            c.tile_begin = tiles;
            tiles += (c.t.n_ado > 1) ? c.n_tiles : 0;
            maxN = std::max(maxN, c.t.N);
            maxW = std::max(maxW, c.t.W);
            maxD = std::max(maxD, c.t.D);
            jobs_stage[off++] = c;
        }
        g.tiles = tiles;
        // the launch sizes LDS for the largest N, W and D of the group
        g.sizing.t.N = maxN;
        g.sizing.t.W = maxW;
        g.sizing.t.D = maxD;
        g.sizing.herm = g.herm;
        g.sizing.lds_bytes = (uint32_t)fma_bytes;
        g.sizing.any_complex_h = any_hc;
        if (g.nb == 0) g.sizing.t.h_complex = 1;  // selects the FMA path for any N
        if (g.solo) {
            g.sizing = *kv.second.front();  // the job itself, launched alone
            g.tiles = g.sizing.t.n_ado > 1 ? g.sizing.n_tiles : 0;
        }
        groups.push_back(g);
    }
    hipError_t e = hipMemcpyAsync(jobs_dev, jobs_stage, n * sizeof(heom::Job),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && n_bjobs)
        e = hipMemcpyAsync(bjobs_dev, bjobs_stage, n_bjobs * sizeof(heom::BlockJob),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(stage_ev, stream);
    if (e != hipSuccess) {
        fail_all("job table upload", e);
        return false;
    }
    dirty = false;
    return true;
}

bool heom_server::launch_macro_step() {
    heom::StageSpec sp[4];
    heom::rk4_stage_specs(sp);
    hipError_t e = hipSuccess;
    if (macro >= 2) e = hipEventSynchronize(step_ev[macro % 2]);  // at most two steps in flight
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
        for (const Group& g : groups) {
            e = heom::launch_stage(g.sizing, g.solo ? nullptr : jobs_dev + g.job_off,
                                   g.solo ? 0 : g.n_jobs, g.tiles, g.precision, sp[k], stream);
            if (e != hipSuccess) break;
        }
        // every coherence-block request in one launch per stage
        if (e == hipSuccess) e = heom::launch_block_stage_batched(bjobs_dev, n_bjobs, btotal, sp[k], stream);
    }
    if (e == hipSuccess) e = heom::launch_block_record_batched(bjobs_dev, n_bjobs, stream);
    if (e == hipSuccess) e = hipEventRecord(step_ev[macro % 2], stream);
    if (e != hipSuccess) {
        fail_all("macro-step launch", e);
        return false;
    }
    ++macro;
    return true;
}

void heom_server::start_drain(Req* r) {
    char* pin = pinned + r->pinned_off;
    const int N = r->info.n_states;
    const size_t NN = (size_t)N * N;
    size_t poff = 0;
    hipError_t e = hipSuccess;
    if (r->block) {
        e = hipMemcpyAsync(pin + r->bpin_rec(), r->brec, (size_t)r->n_rec * 6 * 8,
                           hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pin + r->bpin_status(), r->bstatus, 4, hipMemcpyDeviceToHost, stream);
    }
    for (int k = 0; !r->block && k < r->n_runs && e == hipSuccess; ++k) {
        poff += align256(NN * 16) + align256(heom::control_bytes(N));
        const heom::Job& j = r->jobs[k];
        const size_t rec_bytes = (size_t)r->n_rec * r->rd * 8;
        e = hipMemcpyAsync(pin + poff, j.records, rec_bytes, hipMemcpyDeviceToHost, stream);
        poff += align256(rec_bytes);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pin + poff, j.status, 4, hipMemcpyDeviceToHost, stream);
        poff += 256;
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r->done_ev, stream);
    if (e != hipSuccess) {
        finish(r, HEOM_E_DEVICE);
        fail_all_locked("result copy", e);
        return;
    }
    r->phase = Req::DRAINING;
    draining.push_back(r);
}

void heom_server::finish_draining() {
    std::lock_guard<std::mutex> lk(mu);
    for (auto it = draining.begin(); it != draining.end();) {
        Req* r = *it;
        if (hipEventQuery(r->done_ev) != hipSuccess) {
            ++it;
            continue;
        }
        const char* pin = pinned + r->pinned_off;
        const int N = r->info.n_states;
        const size_t NN = (size_t)N * N;
        const size_t rec_doubles = (size_t)r->n_rec * r->rd;
        r->records.assign(rec_doubles * r->n_runs, 0.0);
        size_t poff = 0;
        int32_t bad = 0;
        if (r->block) {
            // the full form's dipole records [Re P, Im P, Re Tr, Im Tr]; the
            // (e, g) block has no diagonal element, so the trace is 0
            const double* rec6 = reinterpret_cast<const double*>(pin + r->bpin_rec());
            for (int k = 0; k < r->n_runs; ++k)
                for (int64_t q = 0; q < r->n_rec; ++q) {
                    r->records[rec_doubles * k + q * r->rd] = rec6[6 * q + 2 * k];
                    r->records[rec_doubles * k + q * r->rd + 1] = rec6[6 * q + 2 * k + 1];
                }
            std::memcpy(&bad, pin + r->bpin_status(), 4);
        }
        for (int k = 0; !r->block && k < r->n_runs; ++k) {
            poff += align256(NN * 16) + align256(heom::control_bytes(N));
            std::memcpy(r->records.data() + rec_doubles * k, pin + poff, rec_doubles * 8);
            poff += align256(rec_doubles * 8);
            int32_t st;
            std::memcpy(&st, pin + poff, 4);
            bad |= st;
            poff += 256;
        }
        release_resources(r);
        finish(r, r->cancel ? HEOM_E_CANCELLED : (bad ? HEOM_E_NUMERIC : HEOM_OK));
        it = draining.erase(it);
    }
}

void heom_server::run() {
    (void)hipSetDevice(device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop) break;
            if (active.empty() && draining.empty())
                cv_work.wait(lk, [&] { return stop || !pending.empty(); });
            if (stop) break;
        }
        finish_draining();
        admit();
        {
            std::lock_guard<std::mutex> lk(mu);
            if (stop) break;
            // cancelled active requests leave at this step boundary
            for (auto it = active.begin(); it != active.end();) {
                if ((*it)->cancel) {
                    start_drain(*it);
                    it = active.erase(it);
                    dirty = true;
                } else {
                    ++it;
                }
            }
        }
        if (active.empty()) {
            if (!draining.empty()) std::this_thread::yield();
            continue;
        }
        if (dirty && !rebuild()) break;
        if (!launch_macro_step()) break;
        std::lock_guard<std::mutex> lk(mu);
        for (auto it = active.begin(); it != active.end();) {
            Req* r = *it;
            if (++r->steps_done >= r->n_steps) {
                start_drain(r);
                it = active.erase(it);
                dirty = true;
            } else {
                ++it;
            }
        }
    }
    // wait for the device before the arena is handed back
    (void)hipStreamSynchronize(stream);
}

extern "C" {

heom_status heom_server_create(void* arena_dev, size_t arena_bytes, int32_t max_active,
                               void* stream, heom_server** out) {
    if (!out) return srv_fail(HEOM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!arena_dev || reinterpret_cast<uintptr_t>(arena_dev) % 256)
        return srv_fail(HEOM_E_INVAL, "arena must be non-NULL and 256-byte aligned");
    if (max_active < 1 || max_active > 4096) return srv_fail(HEOM_E_INVAL, "max_active outside 1..4096");
    auto* s = new heom_server();
    s->arena = static_cast<char*>(arena_dev);
    s->max_active = max_active;
    s->stream = static_cast<hipStream_t>(stream);
    s->jobs_cap = (size_t)max_active * kMaxRuns;
    const size_t table_bytes = job_table_bytes(s->jobs_cap, max_active);
    if (arena_bytes <= table_bytes) {
        delete s;
        return srv_fail(HEOM_E_NOMEM, "arena smaller than the job table");
    }
    s->jobs_dev = reinterpret_cast<heom::Job*>(s->arena);
    s->bjobs_dev = reinterpret_cast<heom::BlockJob*>(s->arena + align256(s->jobs_cap * sizeof(heom::Job)));
    s->arena_bytes = arena_bytes;
    // the job table occupies the start of the arena
    s->arena_alloc.reset(arena_bytes);
    size_t off;
    s->arena_alloc.alloc(table_bytes, &off);
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->pinned), kPinnedPool, 0);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->jobs_stage), table_bytes, 0);
    if (e == hipSuccess)
        s->bjobs_stage = reinterpret_cast<heom::BlockJob*>(reinterpret_cast<char*>(s->jobs_stage) +
                                                            align256(s->jobs_cap * sizeof(heom::Job)));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->stage_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->step_ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->step_ev[1], hipEventDisableTiming);
    if (e != hipSuccess) {
        if (s->pinned) (void)hipHostFree(s->pinned);
        if (s->jobs_stage) (void)hipHostFree(s->jobs_stage);
        delete s;
        return srv_fail(HEOM_E_DEVICE, std::string("server setup: ") + hipGetErrorString(e));
    }
    s->pinned_alloc.reset(kPinnedPool);
    s->thr = std::thread([s] { s->run(); });
    *out = s;
    return HEOM_OK;
}

// A dipole request the coherence-block form can run: at most three
// directions, the ground state without a bath and without coupling, and
// initial states zero outside column g (rows != g).  The block step check
// comes after, on the block problem.
static bool block_eligible(const heom_request& q, int N) {
    if (q.obs.kind != HEOM_OBS_DIPOLE || q.n_runs > 3 || N < 2 || N - 1 > 64) return false;
    const int g = q.obs.ground;
    const double* H = q.problem.h_re_cm;
    for (int a = 0; a < N; ++a)
        if (a != g && (H[(size_t)a * N + g] != 0.0 || H[(size_t)g * N + a] != 0.0)) return false;
    if (q.problem.h_im_cm)
        for (size_t e = 0; e < (size_t)N * N; ++e)
            if (q.problem.h_im_cm[e] != 0.0) return false;
    for (int b = 0; b < q.problem.n_baths; ++b)
        if (q.problem.baths[b].state == g) return false;
    const size_t NN = (size_t)N * N;
    for (int k = 0; k < q.n_runs; ++k)
        for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b) {
                if (b == g && a != g) continue;
                const double* z = q.rho0 + 2 * (NN * k + (size_t)a * N + b);
                if (z[0] != 0.0 || z[1] != 0.0) return false;
            }
    return true;
}

heom_status heom_submit(heom_server* s, const heom_request* q, uint64_t* ticket) {
    if (!s || !q || !ticket) return srv_fail(HEOM_E_INVAL, "NULL argument");
    if (q->problem.precision == HEOM_FP32_HERM)
        return srv_fail(HEOM_E_INVAL, "the server takes HEOM_FP64 and HEOM_FP32_MIXED requests");
    heom_info info;
    heom_status st = heom_plan(&q->problem, &info);
    if (st != HEOM_OK) return srv_fail(st, heom_last_error());
    if (q->n_runs < 1 || q->n_runs > kMaxRuns) return srv_fail(HEOM_E_INVAL, "n_runs outside 1..8");
    if (q->n_steps < 1 || q->record_every < 1) return srv_fail(HEOM_E_INVAL, "n_steps or record_every < 1");
    if (!(q->dt_fs > 0.0) || !std::isfinite(q->dt_fs)) return srv_fail(HEOM_E_INVAL, "dt must be > 0");
    if (!q->rho0) return srv_fail(HEOM_E_INVAL, "rho0 is NULL");
    const int kind = q->obs.kind;
    if (kind != HEOM_OBS_POPULATION && kind != HEOM_OBS_DIPOLE)
        return srv_fail(HEOM_E_INVAL, "observable kind unknown");
    const int N = info.n_states;
    if (kind == HEOM_OBS_DIPOLE && (!q->obs.mu || q->obs.ground < 0 || q->obs.ground >= N))
        return srv_fail(HEOM_E_INVAL, "dipole observable needs mu and a ground index in range");
    double rate = 0.0;
    heom::problem_rate_bound(&q->problem, &rate);
    if (q->dt_fs * rate > heom::rk4_real_limit())
        return srv_fail(HEOM_E_UNSTABLE, "dt times the rate bound exceeds the RK4 interval");

    auto r = std::make_unique<Req>();
    const size_t NN = (size_t)N * N;
    r->h_re.assign(q->problem.h_re_cm, q->problem.h_re_cm + NN);
    if (q->problem.h_im_cm) r->h_im.assign(q->problem.h_im_cm, q->problem.h_im_cm + NN);
    r->baths.assign(q->problem.baths, q->problem.baths + q->problem.n_baths);
    r->prob = q->problem;
    r->prob.h_re_cm = r->h_re.data();
    r->prob.h_im_cm = q->problem.h_im_cm ? r->h_im.data() : nullptr;
    r->prob.baths = r->baths.data();
    r->n_runs = q->n_runs;
    r->record_every = q->record_every;
    r->kind = kind;
    r->ground = kind == HEOM_OBS_DIPOLE ? q->obs.ground : 0;
    r->hermitian = q->hermitian ? 1 : 0;
    r->n_steps = q->n_steps;
    r->dt = q->dt_fs;
    r->rho0.assign(q->rho0, q->rho0 + 2 * NN * q->n_runs);
    if (kind == HEOM_OBS_DIPOLE) r->mu.assign(q->obs.mu, q->obs.mu + (size_t)N * q->n_runs);
    r->info = info;
    r->n_rec = heom_record_count(q->n_steps, q->record_every);
    r->rd = heom_record_doubles(N, kind);
    r->work_bytes = align256(heom_propagate_work_bytes(&info, q->n_steps, q->record_every, kind));
    r->state_bytes = align256(info.sigma0_bytes) + align256(std::max<size_t>(info.rest_bytes, 1));
    r->footprint = align256(info.tables_bytes) + (size_t)q->n_runs * (r->state_bytes + r->work_bytes);
    r->pinned_bytes = (size_t)q->n_runs * (align256(NN * 16) + align256(heom::control_bytes(N)) +
                                           align256((size_t)r->n_rec * r->rd * 8) + 256);
    if (q->form != HEOM_FORM_AUTO && q->form != HEOM_FORM_FULL)
        return srv_fail(HEOM_E_INVAL, "form unknown");
    if (q->form == HEOM_FORM_AUTO && block_eligible(*q, N)) {
        // the excited block (rows and columns != g) with the ground energy
        // subtracted, the baths renumbered, and the (e, g) columns of the
        // initial states as the start of the three directions
        const int g = q->obs.ground, bN = N - 1;
        r->bN = bN;
        r->bh_re.resize((size_t)bN * bN);
        for (int a = 0, i = 0; a < N; ++a) {
            if (a == g) continue;
            for (int b = 0, j = 0; b < N; ++b) {
                if (b == g) continue;
                r->bh_re[(size_t)i * bN + j] =
                    q->problem.h_re_cm[(size_t)a * N + b] - (a == b ? q->problem.h_re_cm[(size_t)g * N + g] : 0.0);
                ++j;
            }
            ++i;
        }
        r->bbaths = r->baths;
        for (heom_bath& b : r->bbaths) b.state -= b.state > g ? 1 : 0;
        r->bprob = r->prob;
        r->bprob.n_states = bN;
        r->bprob.h_re_cm = r->bh_re.data();
        r->bprob.h_im_cm = nullptr;
        r->bprob.baths = r->bbaths.data();
        heom_info bi;
        if (heom_plan(&r->bprob, &bi) == HEOM_OK && heom::block_step_ok(&r->bprob, q->dt_fs)) {
            r->block = true;
            r->binfo = bi;
            r->bobs.assign((size_t)3 * bN, 0.0);
            r->bstart.assign((size_t)bN * 3 * 2, 0.0);
            for (int k = 0; k < q->n_runs; ++k)
                for (int a = 0, i = 0; a < N; ++a) {
                    if (a == g) continue;
                    r->bobs[(size_t)k * bN + i] = q->obs.mu[(size_t)k * N + a];
                    const double* z = q->rho0 + 2 * (NN * k + (size_t)a * N + g);
                    r->bstart[2 * ((size_t)i * 3 + k)] = z[0];
                    r->bstart[2 * ((size_t)i * 3 + k) + 1] = z[1];
                    ++i;
                }
            r->bstate_bytes = align256((size_t)bi.n_ado * bN * 3 * 16);
            r->bwork_bytes = align256(heom_block_work_bytes(&bi, q->n_steps, q->record_every));
            r->footprint = align256(bi.tables_bytes) + r->bstate_bytes + r->bwork_bytes +
                           align256((size_t)3 * bN * 8);
            r->pinned_bytes = r->bpin_status() + 256;
        }
    }
    const size_t usable = s->arena_bytes - job_table_bytes(s->jobs_cap, s->max_active);
    if (r->footprint > usable || r->pinned_bytes > kPinnedPool)
        return srv_fail(HEOM_E_NOMEM, "request can never fit the arena");
    r->t_submit = heom::monotonic_seconds();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return srv_fail(s->fatal != HEOM_OK ? s->fatal : HEOM_E_INVAL,
                                 s->fatal_msg.empty() ? "server stopped" : s->fatal_msg);
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->all[r->ticket] = std::move(r);
    s->cv_work.notify_all();
    return HEOM_OK;
}

static void fill_result(const Req* r, heom_result* out) {
    out->status = r->status;
    out->n_records = r->n_rec;
    out->record_doubles = r->rd;
    out->records = r->phase == Req::DONE && !r->records.empty() ? r->records.data() : nullptr;
    out->t_submit_s = r->t_submit;
    out->t_admit_s = r->t_admit;
    out->t_finish_s = r->t_finish;
    out->form = r->block ? HEOM_FORM_BLOCK : HEOM_FORM_FULL;
}

heom_status heom_poll(heom_server* s, uint64_t ticket, heom_result* out) {
    if (!s) return srv_fail(HEOM_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return srv_fail(HEOM_E_NOTFOUND, "unknown ticket");
    const Req* r = it->second.get();
    if (out) fill_result(r, out);
    return r->phase == Req::DONE ? r->status : HEOM_PENDING;
}

heom_status heom_wait(heom_server* s, uint64_t ticket, double timeout_s, heom_result* out) {
    if (!s) return srv_fail(HEOM_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return srv_fail(HEOM_E_NOTFOUND, "unknown ticket");
    Req* r = it->second.get();
    auto done = [&] { return r->phase == Req::DONE; };
    if (timeout_s < 0)
        s->cv_done.wait(lk, done);
    else
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    if (out) fill_result(r, out);
    return r->phase == Req::DONE ? r->status : HEOM_PENDING;
}

heom_status heom_cancel(heom_server* s, uint64_t ticket) {
    if (!s) return srv_fail(HEOM_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return srv_fail(HEOM_E_NOTFOUND, "unknown ticket");
    it->second->cancel = true;
    s->cv_work.notify_all();
    return HEOM_OK;
}

heom_status heom_release(heom_server* s, uint64_t ticket) {
    if (!s) return srv_fail(HEOM_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return srv_fail(HEOM_E_NOTFOUND, "unknown ticket");
    if (it->second->phase != Req::DONE) return srv_fail(HEOM_E_INVAL, "request not finished");
    s->all.erase(it);
    return HEOM_OK;
}

heom_status heom_server_set_log(heom_server* s, const char* path) {
    if (!s) return srv_fail(HEOM_E_INVAL, "server is NULL");
    std::FILE* f = nullptr;
    if (path && !(f = std::fopen(path, "a"))) return srv_fail(HEOM_E_INVAL, "cannot open the log file");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->log) std::fclose(s->log);
    s->log = f;
    return HEOM_OK;
}

heom_status heom_server_destroy(heom_server* s) {
    if (!s) return HEOM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->thr.joinable()) s->thr.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->all) {
        Req* r = kv.second.get();
        s->release_resources(r);
    }
    if (s->pinned) (void)hipHostFree(s->pinned);
    if (s->jobs_stage) (void)hipHostFree(s->jobs_stage);
    if (s->stage_ev) (void)hipEventDestroy(s->stage_ev);
    for (auto& e : s->step_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->log) std::fclose(s->log);
    delete s;
    return HEOM_OK;
}

}  // extern "C"
