// Serving of sweep jobs (include/spegg.h, "serving"): a first-fit arena
// over the caller's device memory, a FIFO of waiting jobs, and continuous
// batching -- between steps finished jobs leave and waiting jobs join.
// Each resident job is one population handle carved from the arena, on one
// of the server's streams (the least loaded at admission), so the kernels
// of different jobs overlap on the device; a step replays each job's
// generation graphs on its stream and then waits for every stream.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "spegg.h"
#include "spegg_internal.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size): free blocks keyed by offset,
// neighbours merged on release.
class Arena {
  public:
    explicit Arena(size_t size) : size_(size) {
        if (size > 0) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t used() const { return used_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &f : free_) m = f.second > m ? f.second : m;
        return m;
    }
    size_t size() const { return size_; }

  private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Job {
    uint64_t id = 0;
    std::vector<spegg_rep_desc> reps;
    std::vector<std::vector<int8_t>> effects;  // owned copies behind reps[i].effects
    uint32_t remaining = 0;
    size_t bytes = 0, off = 0;
    uint32_t lane = 0;   // stream index
    double load = 0.0;   // genotype-locus updates per generation at admission
    spegg_pop *pop = nullptr;
};

constexpr uint32_t kMaxStreams = 8;

spegg_status sfail(spegg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    spegg::set_last_error(buf);
    return st;
}

}  // namespace

struct spegg_server {
    uint8_t *base = nullptr;
    std::vector<hipStream_t> lanes;  // lanes[0] is the caller's stream
    std::vector<double> lane_load;
    Arena arena{0};
    std::deque<Job> waiting;
    std::vector<Job> resident;
    std::vector<uint64_t> finished;  // not yet polled
    std::unordered_map<uint64_t, std::vector<spegg_rep_stats>> results;
    bool errored = false;

    bool known(uint64_t id) const {
        for (const Job &j : waiting)
            if (j.id == id) return true;
        for (const Job &j : resident)
            if (j.id == id) return true;
        return results.count(id) != 0;
    }
};

namespace {

// Report a failure of the library call that returned st (its message is
// in spegg_last_error), keeping the server usable unless the device failed.
spegg_status pass_on(spegg_server *s, spegg_status st, const char *what) {
    if (st == SPEGG_E_DEVICE || st == SPEGG_E_STATE) s->errored = true;
    const std::string inner = spegg_last_error();
    return sfail(st, "%s: %s", what, inner.c_str());
}

void drop(spegg_server *s, Job &j) {
    if (j.pop) spegg_pop_destroy(j.pop);
    j.pop = nullptr;
    s->arena.release(j.off, j.bytes);
    s->lane_load[j.lane] -= j.load;
}

hipError_t sync_lanes(spegg_server *s) {
    hipError_t first = hipSuccess;
    for (hipStream_t st : s->lanes) {
        const hipError_t e = hipStreamSynchronize(st);
        if (first == hipSuccess) first = e;
    }
    return first;
}

}  // namespace

extern "C" {

spegg_status spegg_server_create(void *device_mem, size_t device_bytes, void *hip_stream, uint32_t n_streams,
                                 spegg_server **out) {
    if (!out) return sfail(SPEGG_E_INVALID, "server_create: null output pointer");
    *out = nullptr;
    if (!device_mem || ((uintptr_t)device_mem & (kAlign - 1)) != 0)
        return sfail(SPEGG_E_NOMEM, "server_create: the arena must be a non-null, %zu-byte aligned pointer", kAlign);
    if (n_streams < 1 || n_streams > kMaxStreams)
        return sfail(SPEGG_E_INVALID, "server_create: n_streams %u outside 1..%u", n_streams, kMaxStreams);
    spegg_server *s = new spegg_server();
    s->base = (uint8_t *)device_mem;
    s->arena = Arena(device_bytes & ~(kAlign - 1));
    s->lanes.push_back((hipStream_t)hip_stream);
    hipError_t e = hipSuccess;
    if (n_streams > 1) e = hipStreamSynchronize((hipStream_t)hip_stream);
    for (uint32_t k = 1; k < n_streams && e == hipSuccess; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreate(&st);  // default priority
        if (e == hipSuccess) s->lanes.push_back(st);
    }
    if (e != hipSuccess) {
        spegg_server_destroy(s);
        return sfail(SPEGG_E_DEVICE, "server_create: %s", hipGetErrorString(e));
    }
    s->lane_load.assign(s->lanes.size(), 0.0);
    *out = s;
    return SPEGG_OK;
}

spegg_status spegg_server_submit(spegg_server *s, uint64_t job_id, const spegg_rep_desc *reps, uint32_t n_reps,
                                 uint32_t n_generations) {
    if (!s) return sfail(SPEGG_E_INVALID, "null server");
    if (s->errored) return sfail(SPEGG_E_STATE, "server is errored by an earlier device failure");
    if (!reps || n_reps == 0 || n_generations == 0)
        return sfail(SPEGG_E_INVALID, "server_submit: need replicates and at least one generation");
    if (s->known(job_id)) return sfail(SPEGG_E_INVALID, "server_submit: job %llu is already known",
                                       (unsigned long long)job_id);
    const size_t bytes = spegg_footprint(reps, n_reps);
    if (bytes == 0) {
        const std::string inner = spegg_last_error();
        return sfail(SPEGG_E_INVALID, "server_submit: %s", inner.c_str());
    }
    if (align_up(bytes) > s->arena.size())
        return sfail(SPEGG_E_NOMEM, "server_submit: job %llu needs %zu bytes, the arena holds %zu",
                     (unsigned long long)job_id, bytes, s->arena.size());
    Job j;
    j.id = job_id;
    j.reps.assign(reps, reps + n_reps);
    j.effects.resize(n_reps);
    for (uint32_t i = 0; i < n_reps; ++i)
        if (reps[i].effects) {
            j.effects[i].assign(reps[i].effects, reps[i].effects + reps[i].n_loci);
            j.reps[i].effects = j.effects[i].data();
        }
    j.remaining = n_generations;
    j.bytes = bytes;
    s->waiting.push_back(std::move(j));
    return SPEGG_OK;
}

spegg_status spegg_server_step(spegg_server *s, uint32_t n_generations, uint32_t *n_resident, uint32_t *n_waiting) {
    if (!s) return sfail(SPEGG_E_INVALID, "null server");
    if (s->errored) return sfail(SPEGG_E_STATE, "server is errored by an earlier device failure");
    // admission: oldest first, while the oldest fits
    while (!s->waiting.empty()) {
        Job &j = s->waiting.front();
        size_t off;
        if (!s->arena.alloc(j.bytes, &off)) break;
        j.off = off;
        j.lane = 0;
        for (uint32_t k = 1; k < s->lanes.size(); ++k)
            if (s->lane_load[k] < s->lane_load[j.lane]) j.lane = k;
        j.load = 0.0;
        for (const auto &r : j.reps) j.load += (double)r.n0 * r.n_patches * r.n_loci;
        const spegg_status st = spegg_pop_create(j.reps.data(), (uint32_t)j.reps.size(), s->base + off,
                                                 align_up(j.bytes), s->lanes[j.lane], &j.pop);
        if (st != SPEGG_OK) {
            s->arena.release(off, j.bytes);
            return pass_on(s, st, "admitting a job");
        }
        s->lane_load[j.lane] += j.load;
        for (auto &r : j.reps) r.effects = nullptr;  // copied into the job's tables
        j.effects.clear();
        s->resident.push_back(std::move(j));
        s->waiting.pop_front();
    }
    if (n_resident) *n_resident = (uint32_t)s->resident.size();
    if (n_waiting) *n_waiting = (uint32_t)s->waiting.size();
    if (n_generations == 0 || s->resident.empty()) return SPEGG_OK;
    for (Job &j : s->resident) {
        const uint32_t k = j.remaining < n_generations ? j.remaining : n_generations;
        const spegg_status st = spegg_step_generations(j.pop, k);
        if (st != SPEGG_OK) return pass_on(s, st, "stepping a job");
        j.remaining -= k;
    }
    const hipError_t e = sync_lanes(s);
    if (e != hipSuccess) {
        s->errored = true;
        return sfail(SPEGG_E_DEVICE, "server_step: %s", hipGetErrorString(e));
    }
    // retire finished jobs, in residence order
    std::vector<Job> keep;
    keep.reserve(s->resident.size());
    for (Job &j : s->resident) {
        if (j.remaining > 0) {
            keep.push_back(std::move(j));
            continue;
        }
        std::vector<spegg_rep_stats> res(j.reps.size());
        const spegg_status st = spegg_stats(j.pop, res.data(), (uint32_t)res.size());
        if (st != SPEGG_OK) return pass_on(s, st, "reading a finished job");
        s->results[j.id] = std::move(res);
        s->finished.push_back(j.id);
        drop(s, j);
    }
    s->resident = std::move(keep);
    return SPEGG_OK;
}

spegg_status spegg_server_poll(spegg_server *s, uint64_t *job_ids, uint32_t cap, uint32_t *n_out) {
    if (!s || !n_out || (cap && !job_ids)) return sfail(SPEGG_E_INVALID, "server_poll: null argument");
    const uint32_t n = (uint32_t)s->finished.size() < cap ? (uint32_t)s->finished.size() : cap;
    for (uint32_t i = 0; i < n; ++i) job_ids[i] = s->finished[i];
    s->finished.erase(s->finished.begin(), s->finished.begin() + n);
    *n_out = n;
    return SPEGG_OK;
}

spegg_status spegg_server_result(spegg_server *s, uint64_t job_id, spegg_rep_stats *host_out, uint32_t n) {
    if (!s || !host_out) return sfail(SPEGG_E_INVALID, "server_result: null argument");
    auto it = s->results.find(job_id);
    if (it == s->results.end())
        return sfail(SPEGG_E_INVALID, "server_result: job %llu has no unread result", (unsigned long long)job_id);
    if (n != it->second.size())
        return sfail(SPEGG_E_INVALID, "server_result: job %llu has %zu replicates", (unsigned long long)job_id,
                     it->second.size());
    std::memcpy(host_out, it->second.data(), sizeof(spegg_rep_stats) * n);
    s->results.erase(it);
    return SPEGG_OK;
}

spegg_status spegg_server_usage(spegg_server *s, size_t *used, size_t *largest_free) {
    if (!s) return sfail(SPEGG_E_INVALID, "null server");
    if (used) *used = s->arena.used();
    if (largest_free) *largest_free = s->arena.largest_free();
    return SPEGG_OK;
}

void spegg_server_destroy(spegg_server *s) {
    if (!s) return;
    (void)sync_lanes(s);
    for (Job &j : s->resident) drop(s, j);
    for (size_t k = 1; k < s->lanes.size(); ++k) (void)hipStreamDestroy(s->lanes[k]);
    delete s;
}

}  // extern "C"
