// Serving of sweep jobs (include/spegg.h, "serving"): a first-fit arena
// over the caller's device memory, a FIFO of waiting jobs, and continuous
// batching -- between steps finished jobs leave and waiting jobs join.
// Each resident job is one population handle carved from the arena, on one
// of the server's streams (the least loaded at admission), so the kernels
// of different jobs overlap on the device.  A step enqueues each job's
// generations, and a finishing job's census is copied into pinned host
// memory behind its last generation; the step then waits only for the
// previous step's work, so the device runs one step while the host admits
// and retires around the next.
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
    std::vector<std::vector<double>> linkage;  // owned copies behind reps[i].linkage
    std::vector<spegg_ecology> ecology;        // owned copies behind reps[i].ecology
    std::vector<spegg_physiology> physiology;  // owned copies behind reps[i].physiology
    uint32_t remaining = 0;
    size_t bytes = 0, off = 0;
    uint32_t lane = 0;   // stream index
    double load = 0.0;   // genotype-locus updates per generation at admission
    spegg_pop *pop = nullptr;
    bool keep = false;        // hold the population after it finishes (spegg_server_keep)
    bool finishing = false;   // last generation and census copy enqueued
    uint64_t finish_step = 0; // the step that enqueued them
    void *host_states = nullptr;  // pinned copy of the census, filled behind the last generation
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
    std::vector<hipEvent_t> step_ev[2];  // per lane, the end of the last two steps' work
    uint64_t steps = 0;                  // steps that enqueued work
    Arena arena{0};
    std::deque<Job> waiting;
    std::vector<Job> resident;       // admitted, finishing ones included until retired
    std::vector<Job> held;           // finished and kept
    std::vector<uint64_t> finished;  // not yet polled
    std::unordered_map<uint64_t, std::vector<spegg_rep_stats>> results;
    bool errored = false;

    bool known(uint64_t id) const {
        for (const Job &j : waiting)
            if (j.id == id) return true;
        for (const Job &j : resident)
            if (j.id == id) return true;
        for (const Job &j : held)
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

// Release a job whose enqueued work is complete: its handle, pinned census
// copy and arena memory.
void drop(spegg_server *s, Job &j) {
    if (j.pop) spegg::pop_release_done(j.pop);
    j.pop = nullptr;
    if (j.host_states) (void)hipHostFree(j.host_states);
    j.host_states = nullptr;
    s->arena.release(j.off, j.bytes);
    if (!j.keep) s->lane_load[j.lane] -= j.load;
}

// Retire the finishing jobs whose census copies have landed (those that
// finished before step `before`, or all of them): record their results
// and release or hold them.
spegg_status retire(spegg_server *s, uint64_t before, bool all) {
    std::vector<Job> keep;
    keep.reserve(s->resident.size());
    spegg_status bad = SPEGG_OK;
    for (Job &j : s->resident) {
        if (!j.finishing || (!all && j.finish_step >= before)) {
            keep.push_back(std::move(j));
            continue;
        }
        std::vector<spegg_rep_stats> res(j.reps.size());
        const spegg_status st = spegg::pop_results(j.pop, j.host_states, res.data());
        if (st != SPEGG_OK && bad == SPEGG_OK) bad = pass_on(s, st, "reading a finished job");
        s->results[j.id] = std::move(res);
        s->finished.push_back(j.id);
        if (j.keep) {
            s->lane_load[j.lane] -= j.load;  // no more work on its lane
            s->held.push_back(std::move(j));
        } else {
            drop(s, j);
        }
    }
    s->resident = std::move(keep);
    return bad;
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
    j.linkage.resize(n_reps);
    j.ecology.resize(n_reps);
    j.physiology.resize(n_reps);
    for (uint32_t i = 0; i < n_reps; ++i) {
        if (reps[i].physiology) {
            j.physiology[i] = *reps[i].physiology;
            j.reps[i].physiology = &j.physiology[i];
        }
        if (reps[i].effects) {
            j.effects[i].assign(reps[i].effects, reps[i].effects + reps[i].n_loci);
            j.reps[i].effects = j.effects[i].data();
        }
        if (reps[i].linkage) {
            j.linkage[i].assign(reps[i].linkage, reps[i].linkage + (reps[i].n_loci > 1 ? reps[i].n_loci - 1 : 0));
            j.reps[i].linkage = j.linkage[i].data();
        }
        if (reps[i].ecology) {
            j.ecology[i] = *reps[i].ecology;
            j.reps[i].ecology = &j.ecology[i];
        }
    }
    j.remaining = n_generations;
    j.bytes = bytes;
    s->waiting.push_back(std::move(j));
    return SPEGG_OK;
}

spegg_status spegg_server_step(spegg_server *s, uint32_t n_generations, uint32_t *n_resident, uint32_t *n_waiting) {
    if (!s) return sfail(SPEGG_E_INVALID, "null server");
    if (s->errored) return sfail(SPEGG_E_STATE, "server is errored by an earlier device failure");
    if (n_generations == 0) {
        // drain: every enqueued step done, every finished job retired
        const hipError_t e = sync_lanes(s);
        if (e != hipSuccess) {
            s->errored = true;
            return sfail(SPEGG_E_DEVICE, "server_step: %s", hipGetErrorString(e));
        }
        const spegg_status st = retire(s, 0, true);
        if (st != SPEGG_OK) return st;
    }
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
        spegg_status st = spegg_pop_create(j.reps.data(), (uint32_t)j.reps.size(), s->base + off, align_up(j.bytes),
                                           s->lanes[j.lane], &j.pop);
        if (st == SPEGG_OK) {
            const hipError_t e = hipHostMalloc(&j.host_states, spegg::pop_state_bytes(j.pop), hipHostMallocDefault);
            if (e != hipSuccess) {
                j.host_states = nullptr;
                spegg_pop_destroy(j.pop);
                j.pop = nullptr;
                st = sfail(SPEGG_E_DEVICE, "admitting a job: pinned census buffer: %s", hipGetErrorString(e));
            }
        } else {
            st = pass_on(s, st, "admitting a job");
        }
        if (st != SPEGG_OK) {
            s->arena.release(off, j.bytes);
            if (st == SPEGG_E_DEVICE) s->errored = true;
            return st;
        }
        s->lane_load[j.lane] += j.load;
        for (auto &r : j.reps) {  // copied into the job's tables
            r.effects = nullptr;
            r.linkage = nullptr;
            r.ecology = nullptr;
            r.physiology = nullptr;
        }
        j.effects.clear();
        j.linkage.clear();
        j.ecology.clear();
        j.physiology.clear();
        s->resident.push_back(std::move(j));
        s->waiting.pop_front();
    }
    if (n_generations > 0 && !s->resident.empty()) {
        // the step events, made at the first step with work (a server can be
        // created, and take submissions, before any device work)
        hipError_t e = hipSuccess;
        for (int r = 0; r < 2 && e == hipSuccess; ++r)
            while (s->step_ev[r].size() < s->lanes.size() && e == hipSuccess) {
                hipEvent_t ev = nullptr;
                e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (e == hipSuccess) s->step_ev[r].push_back(ev);
            }
        if (e != hipSuccess) {
            s->errored = true;
            return sfail(SPEGG_E_DEVICE, "server_step: events: %s", hipGetErrorString(e));
        }
        const uint64_t step = s->steps++;
        for (Job &j : s->resident) {
            if (j.finishing) continue;
            const uint32_t k = j.remaining < n_generations ? j.remaining : n_generations;
            const spegg_status st = spegg_step_generations(j.pop, k);
            if (st != SPEGG_OK) return pass_on(s, st, "stepping a job");
            j.remaining -= k;
            if (j.remaining == 0) {
                // the census lands in pinned memory behind the last generation
                const hipError_t e = spegg::pop_census_async(j.pop, j.host_states);
                if (e != hipSuccess) {
                    s->errored = true;
                    return sfail(SPEGG_E_DEVICE, "server_step: census of job %llu: %s",
                                 (unsigned long long)j.id, hipGetErrorString(e));
                }
                j.finishing = true;
                j.finish_step = step;
            }
        }
        // this step's work is marked on every lane; the previous step's must
        // be done before the host goes on, so at most two steps are queued
        for (size_t k = 0; k < s->lanes.size() && e == hipSuccess; ++k)
            e = hipEventRecord(s->step_ev[step & 1u][k], s->lanes[k]);
        if (step > 0)
            for (size_t k = 0; k < s->lanes.size() && e == hipSuccess; ++k)
                e = hipEventSynchronize(s->step_ev[(step - 1) & 1u][k]);
        if (e != hipSuccess) {
            s->errored = true;
            return sfail(SPEGG_E_DEVICE, "server_step: %s", hipGetErrorString(e));
        }
        const spegg_status st = retire(s, step, false);
        if (st != SPEGG_OK) return st;
    }
    if (n_resident) *n_resident = (uint32_t)s->resident.size();
    if (n_waiting) *n_waiting = (uint32_t)s->waiting.size();
    return SPEGG_OK;
}

spegg_status spegg_server_keep(spegg_server *s, uint64_t job_id) {
    if (!s) return sfail(SPEGG_E_INVALID, "null server");
    for (Job &j : s->waiting)
        if (j.id == job_id) return j.keep = true, SPEGG_OK;
    for (Job &j : s->resident)
        if (j.id == job_id && !j.finishing) return j.keep = true, SPEGG_OK;
    return sfail(SPEGG_E_INVALID, "server_keep: job %llu is not waiting or running", (unsigned long long)job_id);
}

spegg_status spegg_server_population(spegg_server *s, uint64_t job_id, spegg_pop **out) {
    if (!s || !out) return sfail(SPEGG_E_INVALID, "server_population: null argument");
    *out = nullptr;
    for (Job &j : s->held)
        if (j.id == job_id) return *out = j.pop, SPEGG_OK;
    return sfail(SPEGG_E_INVALID, "server_population: job %llu is not a finished, kept job",
                 (unsigned long long)job_id);
}

spegg_status spegg_server_release(spegg_server *s, uint64_t job_id) {
    if (!s) return sfail(SPEGG_E_INVALID, "null server");
    for (size_t k = 0; k < s->held.size(); ++k)
        if (s->held[k].id == job_id) {
            Job &j = s->held[k];
            // the caller may have enqueued reads on the job's lane
            const hipError_t e = hipStreamSynchronize(s->lanes[j.lane]);
            if (e != hipSuccess) {
                s->errored = true;
                return sfail(SPEGG_E_DEVICE, "server_release: %s", hipGetErrorString(e));
            }
            drop(s, j);
            s->held.erase(s->held.begin() + k);
            return SPEGG_OK;
        }
    return sfail(SPEGG_E_INVALID, "server_release: job %llu is not a finished, kept job", (unsigned long long)job_id);
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
    for (Job &j : s->held) drop(s, j);
    for (int r = 0; r < 2; ++r)
        for (hipEvent_t ev : s->step_ev[r]) (void)hipEventDestroy(ev);
    for (size_t k = 1; k < s->lanes.size(); ++k) (void)hipStreamDestroy(s->lanes[k]);
    delete s;
}

}  // extern "C"
