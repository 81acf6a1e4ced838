// Serving loop over the batched kernels: simulation requests arrive at any
// time, are admitted into a caller-owned device pool when memory and a slot
// are free, advance together (continuous batching: new requests join between
// steps), and are harvested when done.
//
// A step advances the resident lattices on two streams at once.  Lattices on
// the on-chip path (L <= 256 by default) share one batched launch, one block
// per lattice, on the server's stream.  Each gets about the same time on its
// compute unit: a sweep of N sites costs about (N + kSweepCostSites)
// site-update times (a fixed part -- four phase barriers and the latency of
// a phase's dependent LDS reads -- plus a part proportional to N; on MI355X
// the fixed part is worth about 11,000 site updates), so a lattice gets
// max(1, quantum / (N + kSweepCostSites)) sweeps, capped by what the request
// still needs.  Blocks then end together, so a step is not held up by small
// lattices doing many cheap sweeps.  The larger lattices (L = 512) take the
// multi-block word kernel, spread over many compute units, on a second
// stream with its own host thread (the launches of a chunk cost the host about
// 5 us each, and the caller's thread spends most of a step waiting on the
// first stream): while fewer than kSideChunks of its chunks are in flight,
// that thread queues the next one, max(1, quantum / kWordsSweepCostSites)
// sweeps of every such lattice in one launch per phase (a sweep costs about
// kWordsSweepCostSites site-update times of the on-chip kernel whatever their
// number, as the launches are latency-bound), and a finished lattice is
// harvested by a step once the chunk holding its last sweep has completed.  Results are bit-identical to running the same
// request alone: a lattice's chain depends only on its parameters, seed and
// sweep index.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lattice.h"
#include "internal.h"
#include "kernels.h"

using namespace lat;
using namespace lat::detail;

namespace {

constexpr size_t kAlign = 256;
constexpr uint64_t kSweepCostSites = 11000;
// A multi-block sweep of a lattice of L = 512 takes about 22 us on MI355X
// (four dependent phase launches), the time the on-chip kernel needs for
// about 100,000 site updates on its compute unit.  Chunks are sized as if it
// cost half that (twice the sweeps, about 83 a chunk at the default
// quantum), and three are kept in flight: the second stream then depends
// less on how promptly its thread is scheduled.  In alternating 60 s served
// runs this gave a p99 of 0.198-0.220 s against 0.224-0.236 s with two
// chunks of half the length (longer still, 167 sweeps: 0.199 s).
constexpr uint64_t kWordsSweepCostSites = 50000;
// Chunks of the second stream in flight at once: the next ones are queued
// while the first runs, so that stream never waits for the host.
constexpr int kSideChunks = 3;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) of the caller's device pool.
class PoolAllocator {
  public:
    explicit PoolAllocator(size_t size) { free_[0] = size; }

    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }

    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id = 0;
    lat_params params{};
    std::vector<int8_t> init;  // copy of p->init_codes, if any
    uint32_t sweeps = 0, done = 0;
    int32_t status = LAT_REQ_QUEUED;
    int32_t error = 0;  // LAT_E* code of a failed request
    size_t off = 0, bytes = 0;
    lattice *h = nullptr;
    lat_obs obs{};
    uint64_t last_chunk = 0;  // second-stream chunk holding its last sweep (multi-block lattices)
    std::vector<int8_t> final_codes;
    bool keep_state = false;
    double t_submit = 0, t_admit = 0, t_finish = 0;
};

}  // namespace

struct lat_server {
    uint8_t *pool = nullptr;
    size_t pool_bytes = 0;
    size_t obs_off = 0;  // device slot for batched observables (80 B x max_slots)
    int32_t max_slots = 0;
    uint64_t quantum = 0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;               // multi-block lattices advance here, beside the on-chip launch
    hipEvent_t chunk_done[kSideChunks] = {};  // recorded after chunk c in slot c % kSideChunks
    uint64_t chunks_queued = 0, chunks_done = 0;
    // The second stream's own host thread, which enqueues its chunks while
    // the caller's thread waits on the first stream.  mu guards everything
    // below and the requests; the thread sleeps on cv when it has no work.
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    int side_rc = LAT_OK;  // first error of the worker, returned by the next step
    std::string side_msg;
    std::unique_ptr<PoolAllocator> alloc;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> resident;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_id = 1;
    uint64_t steps = 0, site_updates = 0;
};

namespace {

bool server_live(const lat_server *s) { return s != nullptr && s->alloc != nullptr; }

// Admit queued requests in arrival order while a slot and pool memory are
// free (admission stops at the first request that does not fit, so a large
// request is not overtaken indefinitely).
int admit(lat_server *s)
{
    while (!s->queue.empty() && (int32_t)s->resident.size() < s->max_slots) {
        Request &r = *s->reqs[s->queue.front()];
        const size_t sb = lattice_state_bytes(r.params.L, r.params.encoding);
        const size_t cb = lattice_scratch_bytes(r.params.L, r.params.encoding);
        r.bytes = align_up(sb) + cb;
        size_t off;
        if (!s->alloc->alloc(r.bytes, &off)) break;
        r.off = off;
        lat_params p = r.params;
        p.init_codes = r.init.empty() ? nullptr : r.init.data();
        const int rc = lattice_create(&p, s->pool + off, sb, s->pool + off + align_up(sb), cb, s->stream, &r.h);
        if (rc) {
            // the request cannot run (e.g. a HIP error at its set-up): it is
            // reported as failed and the queue moves on, so one bad request
            // never holds up the others
            s->alloc->release(off, r.bytes);
            r.h = nullptr;
            r.status = LAT_REQ_FAILED;
            r.error = rc;
            r.t_finish = now_s();
            s->queue.pop_front();
            continue;
        }
        r.status = LAT_REQ_RESIDENT;
        r.t_admit = now_s();
        s->resident.push_back(r.id);
        s->queue.pop_front();
    }
    return LAT_OK;
}

bool on_chip(const Request &r) { return r.h->path == kPathLds; }

// The second stream's thread.  It keeps up to kSideChunks chunks in flight:
// each holds max(1, quantum / kWordsSweepCostSites) more sweeps of every
// resident multi-block lattice that still needs some, in one launch per
// phase for all of them; a chunk's event marks it complete, and a lattice is
// harvested by the caller's thread once the chunk with its last sweep is.
void side_worker(lat_server *s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        auto has_work = [&] {
            for (uint64_t id : s->resident) {
                const Request &r = *s->reqs[id];
                if (!on_chip(r) && r.done < r.sweeps) return true;
            }
            return false;
        };
        // retire completed chunks; block (without the lock) on the oldest
        // when every slot is taken or there is nothing new to queue
        while (s->chunks_done < s->chunks_queued) {
            hipEvent_t ev = s->chunk_done[s->chunks_done % kSideChunks];
            hipError_t e;
            if (s->chunks_queued - s->chunks_done >= (uint64_t)kSideChunks || !has_work()) {
                lk.unlock();
                e = hipEventSynchronize(ev);
                lk.lock();
            } else {
                e = hipEventQuery(ev);
                if (e == hipErrorNotReady) break;
            }
            if (e != hipSuccess) {
                s->side_rc = hip_fail(e, "server second stream");
                s->side_msg = lattice_last_error();
                return;
            }
            ++s->chunks_done;
        }
        if (s->stop) break;
        std::vector<lattice *> big;
        std::vector<uint32_t> big_sw;
        std::vector<Request *> big_reqs;
        const uint64_t c = s->chunks_queued;  // index of the chunk built now
        for (uint64_t id : s->resident) {
            Request &r = *s->reqs[id];
            if (on_chip(r) || r.done >= r.sweeps) continue;
            const uint64_t N = (uint64_t)r.params.L * r.params.L;
            const uint32_t k = std::min((uint32_t)std::max<uint64_t>(1, s->quantum / kWordsSweepCostSites),
                                        r.sweeps - r.done);
            big.push_back(r.h);
            big_sw.push_back(k);
            big_reqs.push_back(&r);
            r.done += k;
            if (r.done >= r.sweeps) r.last_chunk = c;
            s->site_updates += N * k;
        }
        if (big.empty()) {
            if (s->chunks_done == s->chunks_queued) s->cv.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        lk.unlock();
        // one launch per phase: a cooperative launch beside the on-chip
        // kernels of the first stream could wait for compute units
        int rc = enqueue_offchip_sweeps(big.data(), (int32_t)big.size(), big_sw.data(), 0, s->side,
                                        /*convert=*/true, /*persistent=*/false);
        std::string msg = rc ? lattice_last_error() : "";
        if (rc == LAT_OK) {
            const hipError_t e = hipEventRecord(s->chunk_done[c % kSideChunks], s->side);
            if (e != hipSuccess) {
                rc = hip_fail(e, "server second stream");
                msg = lattice_last_error();
            }
        }
        lk.lock();
        if (rc) {
            s->side_rc = rc;
            s->side_msg = msg;
            return;
        }
        s->chunks_queued = c + 1;
    }
}

// The second stream, its events and its thread, made when a multi-block
// lattice first becomes resident (called with mu held).
int start_side(lat_server *s)
{
    if (s->side) return LAT_OK;
    hipError_t e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
    for (int i = 0; i < kSideChunks && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&s->chunk_done[i], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "lat_server_step: second stream");
    s->worker = std::thread(side_worker, s);
    return LAT_OK;
}

}  // namespace

extern "C" {

int lat_server_create(void *d_pool, size_t pool_bytes, int32_t max_slots, uint64_t quantum_updates,
                      void *hip_stream, lat_server **out)
{
    return guarded("lat_server_create", [&]() -> int {
        if (!out || !d_pool || max_slots <= 0 || quantum_updates == 0) return fail(LAT_EINVAL, "bad server arguments");
        *out = nullptr;
        const size_t obs_bytes = align_up((size_t)max_slots * 80u);
        if (pool_bytes <= obs_bytes) return fail(LAT_ENOMEM, "pool smaller than the observables slot");
        auto *s = new lat_server();
        s->pool = (uint8_t *)d_pool;
        s->pool_bytes = pool_bytes;
        s->obs_off = 0;
        s->max_slots = max_slots;
        s->quantum = quantum_updates;
        s->stream = (hipStream_t)hip_stream;
        s->alloc = std::make_unique<PoolAllocator>(pool_bytes);
        size_t off;
        s->alloc->alloc(obs_bytes, &off);  // offset 0: reserved for observables
        *out = s;
        return LAT_OK;
    });
}

int lat_server_submit(lat_server *s, const lat_params *p, uint32_t sweeps, int32_t keep_state, uint64_t *id)
{
    return guarded("lat_server_submit", [&]() -> int {
        if (!server_live(s)) return fail(LAT_ESTATE, "null or destroyed server");
        if (!p || !id || sweeps == 0) return fail(LAT_EINVAL, "bad request");
        if (p->L > kLdsMaxL || lattice_state_bytes(p->L, p->encoding) == 0)
            return fail(LAT_EINVAL, "served lattices need a valid L <= 512");
        // the checks lattice_create makes, so that a request that could never
        // be admitted is refused here rather than at admission
        int64_t Q = 0, Nc = 0;
        const int rc = validate_params(p, &Q, &Nc);
        if (rc) return rc;
        auto r = std::make_unique<Request>();
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        r->params = *p;
        if (p->init_codes) r->init.assign(p->init_codes, p->init_codes + (size_t)p->L * p->L);
        r->params.init_codes = nullptr;
        r->sweeps = sweeps;
        r->keep_state = keep_state != 0;
        r->t_submit = now_s();
        *id = r->id;
        s->queue.push_back(r->id);
        s->reqs[r->id] = std::move(r);
        return LAT_OK;
    });
}

int lat_server_step(lat_server *s, int32_t *n_finished)
{
    return guarded("lat_server_step", [&]() -> int {
        if (!server_live(s)) return fail(LAT_ESTATE, "null or destroyed server");
        if (n_finished) *n_finished = 0;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->side_rc) return fail(s->side_rc, s->side_msg);
        int rc = admit(s);
        if (rc) return rc;
        if (s->resident.empty()) return LAT_OK;
        bool any_big = false;
        for (uint64_t id : s->resident) any_big = any_big || !on_chip(*s->reqs[id]);
        if (any_big) {
            rc = start_side(s);
            if (rc) return rc;
            s->cv.notify_one();
        }

        // the on-chip lattices: one batched launch on the server's stream
        std::vector<lattice *> hs;
        std::vector<uint32_t> sw;
        for (uint64_t id : s->resident) {
            Request &r = *s->reqs[id];
            if (!on_chip(r) || r.done >= r.sweeps) continue;
            const uint64_t N = (uint64_t)r.params.L * r.params.L;
            const uint32_t want = (uint32_t)std::max<uint64_t>(1, s->quantum / (N + kSweepCostSites));
            const uint32_t k = std::min(want, r.sweeps - r.done);
            hs.push_back(r.h);
            sw.push_back(k);
            r.done += k;
            s->site_updates += N * k;
        }
        // Harvest: on-chip lattices with all their sweeps enqueued (their
        // work is ordered before the harvest on the server's stream), and
        // multi-block ones once the chunk holding their last sweep has
        // completed on the second stream (the worker no longer touches them).
        std::vector<lattice *> fin;
        std::vector<uint64_t> fin_ids;
        std::vector<bool> fin_keep;
        for (uint64_t id : s->resident) {
            const Request &r = *s->reqs[id];
            if (r.done >= r.sweeps && (on_chip(r) || r.last_chunk < s->chunks_done)) {
                fin.push_back(r.h);
                fin_ids.push_back(id);
                fin_keep.push_back(r.keep_state);
            }
        }
        lk.unlock();

        if (!hs.empty()) {
            rc = enqueue_lds_sweeps(hs.data(), (int32_t)hs.size(), sw.data(), 0, s->stream);
            if (rc) return rc;
            ++s->steps;
        }
        std::vector<lat_obs> obs(fin.size());
        std::vector<std::vector<int8_t>> codes(fin.size());
        if (!fin.empty()) {
            rc = lattice_observables_batch(fin.data(), (int32_t)fin.size(), s->pool + s->obs_off,
                                           (size_t)s->max_slots * 80u, obs.data(), s->stream);
            if (rc) return rc;
            for (size_t i = 0; i < fin.size(); ++i) {
                if (!fin_keep[i]) continue;
                codes[i].resize((size_t)fin[i]->L * fin[i]->L);
                rc = lattice_read_state(fin[i], codes[i].data());
                if (rc) return rc;
            }
        }

        lk.lock();
        const double t = now_s();
        for (size_t i = 0; i < fin.size(); ++i) {
            Request &r = *s->reqs[fin_ids[i]];
            r.obs = obs[i];
            r.final_codes = std::move(codes[i]);
            lattice_destroy(r.h);
            r.h = nullptr;
            s->alloc->release(r.off, r.bytes);
            r.status = LAT_REQ_FINISHED;
            r.t_finish = t;
        }
        if (!fin.empty()) {
            std::vector<uint64_t> keep;
            for (uint64_t id : s->resident)
                if (s->reqs[id]->status == LAT_REQ_RESIDENT) keep.push_back(id);
            s->resident = keep;
        }
        if (n_finished) *n_finished = (int32_t)fin.size();
        return LAT_OK;
    });
}

int lat_server_poll(lat_server *s, uint64_t id, lat_request_info *out, int8_t *final_codes)
{
    return guarded("lat_server_poll", [&]() -> int {
        if (!server_live(s)) return fail(LAT_ESTATE, "null or destroyed server");
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end() || !out) return fail(LAT_EINVAL, "unknown request");
        const Request &r = *it->second;
        out->id = r.id;
        out->status = r.status;
        out->error = r.error;
        out->sweeps_total = r.sweeps;
        out->sweeps_done = r.done;
        out->t_submit = r.t_submit;
        out->t_admit = r.t_admit;
        out->t_finish = r.t_finish;
        out->obs = r.obs;
        if (final_codes && r.status == LAT_REQ_FINISHED) {
            if (!r.keep_state) return fail(LAT_EINVAL, "request was submitted without keep_state");
            std::memcpy(final_codes, r.final_codes.data(), r.final_codes.size());
        }
        return LAT_OK;
    });
}

int lat_server_release(lat_server *s, uint64_t id)
{
    return guarded("lat_server_release", [&]() -> int {
        if (!server_live(s)) return fail(LAT_ESTATE, "null or destroyed server");
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end() ||
            (it->second->status != LAT_REQ_FINISHED && it->second->status != LAT_REQ_FAILED))
            return fail(LAT_EINVAL, "not finished");
        s->reqs.erase(it);
        return LAT_OK;
    });
}

int lat_server_stats(lat_server *s, lat_server_counters *out)
{
    return guarded("lat_server_stats", [&]() -> int {
        if (!server_live(s)) return fail(LAT_ESTATE, "null or destroyed server");
        std::lock_guard<std::mutex> lk(s->mu);
        if (!out) return fail(LAT_EINVAL, "null output");
        out->queued = (int32_t)s->queue.size();
        out->resident = (int32_t)s->resident.size();
        out->pool_used = s->alloc->used();
        out->steps = s->steps;
        out->site_updates = s->site_updates;
        return LAT_OK;
    });
}

int lat_server_destroy(lat_server *s)
{
    return guarded("lat_server_destroy", [&]() -> int {
        if (!server_live(s)) return fail(LAT_ESTATE, "null or destroyed server");
        if (s->worker.joinable()) {
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->stop = true;
            }
            s->cv.notify_one();
            s->worker.join();
        }
        hipError_t e = s->side ? hipStreamSynchronize(s->side) : hipSuccess;
        const hipError_t e2 = hipStreamSynchronize(s->stream);
        if (e == hipSuccess) e = e2;
        for (auto &kv : s->reqs)
            if (kv.second->h) lattice_destroy(kv.second->h);
        s->alloc.reset();
        for (hipEvent_t ev : s->chunk_done)
            if (ev) (void)hipEventDestroy(ev);
        if (s->side) (void)hipStreamDestroy(s->side);
        delete s;
        return e == hipSuccess ? LAT_OK : hip_fail(e, "lat_server_destroy");
    });
}

}  // extern "C"
