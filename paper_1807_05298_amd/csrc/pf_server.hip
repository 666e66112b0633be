// Serving loop: continuous batching of many reservoir realisations on one GPU.
//
// The caller hands the server one device arena.  Submitted realisations
// (model + initial state + step schedule, deep-copied at submission) wait in
// a queue.  Each of max_slots worker threads owns a HIP stream; a free
// worker admits the first queued request, in arrival order, whose HBM
// footprint (its pf_workspace_size) fits the arena's free space (first fit;
// a request that does not fit yet lets at most kMaxBypass later ones pass
// before admissions wait for it), creates a simulator on that sub-allocation
// and its stream, runs the schedule with pf_step, records the wall latency
// of every step, then releases the memory and takes the next request.
// Requests that arrive while others run join as soon as a slot and memory
// free up; the work of all active realisations overlaps on the device
// through their streams.  In a fused server the slots are spread over a few
// fusion groups (pf_fuse.hip), each on a stream of its own: the active
// realisations of a group are its members for their steps, their launches
// merged into shared launches, and the groups' streams overlap on the
// device.  Every realisation runs the same kernels with the same arguments
// as when alone, so its results do not depend on the mix.
#include "pf_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

namespace {

// A request at the head of the queue lets at most this many later ones be
// admitted before it (first fit), so a large request is not starved.
constexpr int kMaxBypass = 8;

struct Job {
    uint64_t ticket = 0;
    // owned copies of the request
    pf_grid grid;
    pf_rock rock;
    pf_fluid fluid;
    pf_polymer polymer;
    std::vector<pf_well> wells;
    std::vector<double> poro, kx, ky, kz, P0, S0, C0, Pb0, dts;
    pf_solver_opts opts;
    size_t bytes = 0;
    int bypassed = 0;                // later requests admitted while this one waited at the head
    // results
    int32_t state = 0;               // 0 queued, 1 running, 2 done, 3 failed
    std::vector<double> P, S, C, Pb, latency;
    std::vector<int32_t> newton, lin;
    std::string error;
    double t_submit = 0.0, t_start = 0.0, t_end = 0.0;

    pf_model_desc desc() const {
        pf_model_desc d;
        d.grid = grid;
        d.rock = rock;
        d.rock.poro = poro.data();
        d.rock.kx = kx.data();
        d.rock.ky = ky.data();
        d.rock.kz = kz.data();
        d.fluid = fluid;
        d.polymer = polymer;
        d.n_wells = (int32_t)wells.size();
        d.wells = wells.empty() ? nullptr : wells.data();
        return d;
    }
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with 256-byte granularity.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;      // offset -> length
    void init(size_t n) {
        size = n & ~size_t(255);
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t* off) {
        n = (n + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t o2 = it->first + n;
                free_.erase(it);
                if (rest) free_[o2] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) & ~size_t(255);
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
    size_t largest() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
    size_t total_free() const {
        size_t m = 0;
        for (auto& kv : free_) m += kv.second;
        return m;
    }
};

}  // namespace

struct pf_server {
    char* base = nullptr;
    int device = 0;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv;          // queue / memory / completion changes
    std::deque<std::shared_ptr<Job>> queue;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    int running = 0;
    int peak_running = 0;
    size_t peak_bytes = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    // fused server: fusion groups of the active realisations, each on a stream
    // of its own (slot i belongs to group i % groups)
    std::vector<pf_fusion*> fusion;
    std::vector<hipStream_t> fusion_streams;
};

namespace {

void worker_main(pf_server* sv, int idx) {
    (void)hipSetDevice(sv->device);
    hipStream_t stream = sv->streams[idx];
    for (;;) {
        std::shared_ptr<Job> job;
        size_t off = 0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (;;) {
                if (sv->stop) return;
                if (!sv->queue.empty()) {
                    auto& head = sv->queue.front();
                    if (head->bytes > sv->arena.size) {      // can never fit
                        head->state = 3;
                        head->error = "footprint exceeds the server arena";
                        sv->queue.pop_front();
                        sv->cv.notify_all();
                        continue;
                    }
                    // first fit in arrival order over the queue: a request that does not
                    // fit the free memory yet lets later, smaller ones pass, at most
                    // kMaxBypass times, then admissions wait for it
                    const size_t look = head->bypassed >= kMaxBypass ? 1 : sv->queue.size();
                    for (size_t q = 0; q < look; ++q) {
                        auto& cand = sv->queue[q];
                        if (cand->bytes > sv->arena.size || !sv->arena.alloc(cand->bytes, &off)) continue;
                        job = cand;
                        if (q > 0) head->bypassed++;
                        sv->queue.erase(sv->queue.begin() + (std::ptrdiff_t)q);
                        job->state = 1;
                        sv->running++;
                        sv->peak_running = std::max(sv->peak_running, sv->running);
                        sv->peak_bytes = std::max(sv->peak_bytes, sv->arena.size - sv->arena.total_free());
                        break;
                    }
                    if (job) break;
                }
                sv->cv.wait(lk);
            }
        }
        job->t_start = now_s();
        pf_sim* sim = nullptr;
        const pf_model_desc d = job->desc();
        pf_status st = pf_create(&d, &job->opts, sv->base + off, job->bytes, (void*)stream, &sim);
        if (st == PF_OK)
            st = pf_set_state(sim, job->P0.data(), job->S0.data(), job->C0.data(),
                              job->Pb0.empty() ? nullptr : job->Pb0.data());
        pf_fusion* group = sv->fusion.empty() ? nullptr : sv->fusion[idx % sv->fusion.size()];
        if (st == PF_OK && group) st = pf_fusion_join(group, sim);
        for (size_t k = 0; st == PF_OK && k < job->dts.size(); ++k) {
            pf_step_stats ss;
            const double t0 = now_s();
            st = pf_step(sim, job->dts[k], &ss);
            job->latency.push_back(now_s() - t0);
            job->newton.push_back(ss.newton_its);
            job->lin.push_back(ss.lin_its);
        }
        if (sim && group) {
            const pf_status sl = pf_fusion_leave(sim);
            if (st == PF_OK) st = sl;
        }
        if (st == PF_OK) {
            const int64_t n = (int64_t)d.grid.nx * d.grid.ny * d.grid.nz;
            job->P.resize(n);
            job->S.resize(n);
            job->C.resize(n);
            job->Pb.resize(job->wells.size());
            st = pf_get_state(sim, job->P.data(), job->S.data(), job->C.data(), job->Pb.empty() ? nullptr : job->Pb.data());
        }
        if (st != PF_OK) job->error = pf_last_error();
        if (sim) pf_destroy(sim);
        (void)hipStreamSynchronize(stream);
        job->t_end = now_s();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->arena.release(off, job->bytes);
            job->state = (st == PF_OK) ? 2 : 3;
            sv->running--;
        }
        sv->cv.notify_all();
    }
}

}  // namespace

extern "C" {

pf_status pf_server_create(void* dev_arena, size_t arena_bytes, int32_t max_slots, int32_t fused, pf_server** out) {
    if (!dev_arena || !out || max_slots < 1 || max_slots > 64 || (((uintptr_t)dev_arena) & 255) || fused < 0 ||
        fused > max_slots) {
        pf::set_error("bad server arguments");
        return PF_EINVAL;
    }
    pf_server* sv = new pf_server();
    sv->base = (char*)dev_arena;
    sv->arena.init(arena_bytes);
    if (hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        pf::set_error("hipGetDevice failed");
        return PF_EHIP;
    }
    for (int i = 0; i < max_slots; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : sv->streams) (void)hipStreamDestroy(t);
            delete sv;
            pf::set_error("hipStreamCreate failed");
            return PF_EHIP;
        }
        sv->streams.push_back(s);
    }
    for (int g = 0; g < fused; ++g) {
        hipStream_t fs = nullptr;
        pf_fusion* fg = nullptr;
        if (hipStreamCreateWithFlags(&fs, hipStreamNonBlocking) != hipSuccess ||
            pf_fusion_create((void*)fs, &fg) != PF_OK) {
            if (fs) (void)hipStreamDestroy(fs);
            for (pf_fusion* f : sv->fusion) pf_fusion_destroy(f);
            for (hipStream_t q : sv->fusion_streams) (void)hipStreamDestroy(q);
            for (hipStream_t q : sv->streams) (void)hipStreamDestroy(q);
            delete sv;
            pf::set_error("fusion group set-up failed");
            return PF_EHIP;
        }
        sv->fusion.push_back(fg);
        sv->fusion_streams.push_back(fs);
    }
    for (int i = 0; i < max_slots; ++i) sv->workers.emplace_back(worker_main, sv, i);
    *out = sv;
    return PF_OK;
}

pf_status pf_server_submit(pf_server* sv, const pf_model_desc* d, const pf_solver_opts* o, const double* P0,
                           const double* S0, const double* C0, const double* Pb0, int32_t n_steps,
                           const double* dts, uint64_t* ticket) {
    if (!sv || !d || !o || !P0 || !S0 || !C0 || n_steps < 1 || !dts || !ticket ||
        (d->n_wells > 0 && (!Pb0 || !d->wells))) {
        pf::set_error("bad submit arguments");
        return PF_EINVAL;
    }
    size_t bytes = 0;
    pf_status st = pf_workspace_size(d, o, &bytes);
    if (st != PF_OK) return st;
    auto job = std::make_shared<Job>();
    const int64_t n = (int64_t)d->grid.nx * d->grid.ny * d->grid.nz;
    job->grid = d->grid;
    job->rock = d->rock;
    job->fluid = d->fluid;
    job->polymer = d->polymer;
    job->wells.assign(d->wells, d->wells + d->n_wells);
    job->poro.assign(d->rock.poro, d->rock.poro + n);
    job->kx.assign(d->rock.kx, d->rock.kx + n);
    job->ky.assign(d->rock.ky, d->rock.ky + n);
    job->kz.assign(d->rock.kz, d->rock.kz + n);
    job->P0.assign(P0, P0 + n);
    job->S0.assign(S0, S0 + n);
    job->C0.assign(C0, C0 + n);
    if (d->n_wells > 0) job->Pb0.assign(Pb0, Pb0 + d->n_wells);
    job->dts.assign(dts, dts + n_steps);
    job->opts = *o;
    job->bytes = bytes;
    job->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        job->ticket = sv->next_ticket++;
        sv->jobs[job->ticket] = job;
        sv->queue.push_back(job);
    }
    sv->cv.notify_all();
    *ticket = job->ticket;
    return PF_OK;
}

pf_status pf_server_poll(pf_server* sv, uint64_t ticket, int32_t* state, double* P, double* S, double* C, double* Pb,
                         double* step_latency_s, int32_t* newton_its, double* times) {
    if (!sv || !state) {
        pf::set_error("bad poll arguments");
        return PF_EINVAL;
    }
    std::shared_ptr<Job> job;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->jobs.find(ticket);
        if (it == sv->jobs.end()) {
            pf::set_error("unknown ticket");
            return PF_EINVAL;
        }
        job = it->second;
        *state = job->state;
    }
    if (*state == 3) pf::set_error(job->error);
    if (*state != 2) return PF_OK;
    if (P) std::copy(job->P.begin(), job->P.end(), P);
    if (S) std::copy(job->S.begin(), job->S.end(), S);
    if (C) std::copy(job->C.begin(), job->C.end(), C);
    if (Pb) std::copy(job->Pb.begin(), job->Pb.end(), Pb);
    if (step_latency_s) std::copy(job->latency.begin(), job->latency.end(), step_latency_s);
    if (newton_its) std::copy(job->newton.begin(), job->newton.end(), newton_its);
    if (times) { times[0] = job->t_submit; times[1] = job->t_start; times[2] = job->t_end; }
    return PF_OK;
}

pf_status pf_server_wait(pf_server* sv, uint64_t ticket) {
    if (!sv) return PF_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        bool pending = false;
        if (ticket) {
            auto it = sv->jobs.find(ticket);
            if (it == sv->jobs.end()) {
                pf::set_error("unknown ticket");
                return PF_EINVAL;
            }
            pending = it->second->state < 2;
        } else {
            pending = !sv->queue.empty() || sv->running > 0;
        }
        if (!pending) return PF_OK;
        sv->cv.wait(lk);
    }
}

pf_status pf_server_release(pf_server* sv, uint64_t ticket) {
    if (!sv) {
        pf::set_error("null server");
        return PF_EINVAL;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) {
        pf::set_error("unknown ticket");
        return PF_EINVAL;
    }
    if (it->second->state < 2) {
        pf::set_error("the request is still queued or running");
        return PF_EINVAL;
    }
    sv->jobs.erase(it);
    return PF_OK;
}

pf_status pf_server_info(pf_server* sv, int32_t* queued, int32_t* running, int32_t* peak_running,
                         size_t* peak_bytes, size_t* free_bytes) {
    if (!sv) return PF_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (queued) *queued = (int32_t)sv->queue.size();
    if (running) *running = sv->running;
    if (peak_running) *peak_running = sv->peak_running;
    if (peak_bytes) *peak_bytes = sv->peak_bytes;
    if (free_bytes) *free_bytes = sv->arena.total_free();
    return PF_OK;
}

void pf_server_destroy(pf_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->queue.clear();
    }
    sv->cv.notify_all();
    for (auto& t : sv->workers) t.join();
    for (hipStream_t s : sv->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (pf_fusion* f : sv->fusion) pf_fusion_destroy(f);
    for (hipStream_t q : sv->fusion_streams) {
        (void)hipStreamSynchronize(q);
        (void)hipStreamDestroy(q);
    }
    delete sv;
}

}  // extern "C"
