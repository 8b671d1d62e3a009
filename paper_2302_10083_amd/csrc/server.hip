// Serving: a request loop over one device (declared in include/dqmc.h).
//
// One scheduler thread owns every HIP call of the server.  Each round it
//   1. retires finished work (an event per launch), publishing results;
//   2. admits queued jobs first-fit in arrival order while their footprint
//      fits the free budget (a job that has waited longer than kAgingSeconds
//      at the head of the queue stops others from overtaking it);
//   3. launches: all admitted jobs with n <= kBatchMaxN go into one batch on
//      a free batch slot (the device-planned persistent launch of
//      k_batch.hip), each larger job gets a free slot (stream + context) of
//      its own.
// Device memory is one arena of `budget` bytes allocated when the server is
// created; each admitted job gets one block of its footprint from a host-side
// first-fit allocator (large jobs from the low end, small ones from the high
// end, freed blocks coalesce), so a job that arrives while others run starts
// as soon as a block and a slot are free, without any device allocation, and
// its kernels overlap with the running ones.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "dqmc.h"
#include "launch.h"
#include "h5.h"

using namespace dqmc;

namespace {

constexpr double kAgingSeconds = 0.05;
constexpr uint32_t kBatchSlotJobs = 2048;  // jobs per batch launch

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

uint64_t list_reserve(int n)
{
    const uint64_t all = pow3(n);
    uint64_t r = pow3(n > 3 ? n - 3 : 0) / 16;
    if (r < (1ull << 18)) r = 1ull << 18;
    return r < all ? r : all;
}

uint64_t tt_words_of(int n) { return n <= 5 ? 1 : (1ull << (n - 5)); }
uint64_t state_words_of(int n)
{
    return n > 12 ? (uint64_t)kTileStride * pow3(n - 12) : kBlockWords * pow3(n > 5 ? n - 5 : 0);
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Bytes of a job's arena block: state, list reserve, truth table, count.
uint64_t footprint(int n)
{
    return align256(4 * state_words_of(n)) + align256(8 * list_reserve(n)) + align256(4 * tt_words_of(n)) + 256;
}

enum Phase { kPending, kRunning, kDone, kReleased };

// First-fit allocator over [0, size) with coalescing of freed blocks.
class Arena {
  public:
    void init(uint64_t size)
    {
        free_.clear();
        if (size > 0) free_[0] = size;
    }
    // lowest-addressed (or, from_top, highest-addressed) free block that fits
    bool alloc(uint64_t sz, bool from_top, uint64_t *off)
    {
        if (!from_top) {
            for (auto it = free_.begin(); it != free_.end(); ++it)
                if (it->second >= sz) {
                    *off = it->first;
                    const uint64_t rest = it->second - sz, o = it->first + sz;
                    free_.erase(it);
                    if (rest) free_[o] = rest;
                    return true;
                }
        } else {
            for (auto it = free_.rbegin(); it != free_.rend(); ++it)
                if (it->second >= sz) {
                    const uint64_t o = it->first, len = it->second;
                    *off = o + len - sz;
                    if (len == sz) free_.erase(o);
                    else free_[o] = len - sz;
                    return true;
                }
        }
        return false;
    }
    void release(uint64_t off, uint64_t sz)
    {
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + sz == nx->first) {
            sz += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(off);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                pv->second += sz;
                return;
            }
        }
        free_[off] = sz;
    }

  private:
    std::map<uint64_t, uint64_t> free_;  // offset -> length
};

struct SJob {
    uint64_t id = 0;
    int n = 0;
    Phase phase = kPending;
    int status = DQMC_OK;
    uint32_t *h_tt = nullptr;    // pinned copy of the truth table
    uint64_t *h_count = nullptr; // pinned landing slot for the count
    uint32_t *d_tt = nullptr;
    uint32_t *d_state = nullptr;
    uint64_t *d_list = nullptr;
    uint64_t *d_count = nullptr;
    uint64_t cap = 0;
    uint64_t count = 0;
    uint64_t fp = 0;
    uint64_t off = 0;  // arena block
    double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    dqmc_ctx *ctx = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<uint64_t> jobs;
    // batch slots: job table (pinned staging, device copy) and batch scratch
    dqmc_job *h_jobs = nullptr;
    dqmc_job *d_jobs = nullptr;
    void *d_scratch = nullptr;
    BatchScratch bs{};
};

}  // namespace

struct dqmc_server {
    int device = 0;
    uint64_t budget = 0, used = 0;
    uint8_t *arena_base = nullptr;
    Arena arena;
    std::vector<Slot> big, small;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, SJob> jobs;
    std::deque<uint64_t> queue;
    uint64_t next_id = 1;
    bool stop = false;
    bool stalled = false;  // queued work that cannot be admitted while nothing runs
    double head_since = 0;
    uint64_t head_id = 0;
    std::thread thr;
    char err[256] = {0};
};

namespace {

void free_job_device(dqmc_server *s, SJob &j)
{
    if (j.d_state != nullptr) s->arena.release(j.off, j.fp);
    j.d_tt = nullptr;
    j.d_state = nullptr;
    j.d_list = nullptr;
    j.d_count = nullptr;
}

// Carve a job's buffers out of its arena block and enqueue the upload of its
// truth table on `st`.
bool stage_job(dqmc_server *s, SJob &j, hipStream_t st)
{
    const uint64_t nw = tt_words_of(j.n), sw = state_words_of(j.n);
    j.cap = list_reserve(j.n);
    uint8_t *p = s->arena_base + j.off;
    j.d_state = (uint32_t *)p;
    p += align256(4 * sw);
    j.d_list = (uint64_t *)p;
    p += align256(8 * j.cap);
    j.d_tt = (uint32_t *)p;
    p += align256(4 * nw);
    j.d_count = (uint64_t *)p;
    return hipMemcpyAsync(j.d_tt, j.h_tt, nw * 4, hipMemcpyHostToDevice, st) == hipSuccess;
}

void launch_big(dqmc_server *s, Slot &sl, SJob &j)
{
    sl.busy = true;
    sl.jobs.assign(1, j.id);
    bool ok = stage_job(s, j, sl.stream);
    if (ok)
        ok = dqmc_primes(sl.ctx, j.n, j.d_tt, j.d_state, j.d_list, j.cap, j.d_count, sl.stream) == DQMC_OK;
    if (ok) ok = hipMemcpyAsync(j.h_count, j.d_count, 8, hipMemcpyDeviceToHost, sl.stream) == hipSuccess;
    if (!ok) j.status = DQMC_EDEVICE;
    (void)hipEventRecord(sl.ev, sl.stream);
}

void launch_small(dqmc_server *s, Slot &sl, const std::vector<uint64_t> &ids)
{
    sl.busy = true;
    sl.jobs = ids;
    uint32_t m = 0;
    BatchExpect ex{};  // every staged job is valid: its size is known here
    ex.exact = 1;
    for (uint64_t id : ids) {
        SJob &j = s->jobs[id];
        if (!stage_job(s, j, sl.stream)) {
            j.status = DQMC_EDEVICE;
            continue;
        }
        sl.h_jobs[m++] = dqmc_job{j.n, 0, j.d_tt, j.d_state, j.d_list, j.cap, j.d_count};
        ++ex.hist[j.n];
    }
    bool ok = true;
    if (m > 0) {
        ok = hipMemcpyAsync(sl.d_jobs, sl.h_jobs, m * sizeof(dqmc_job), hipMemcpyHostToDevice, sl.stream) ==
             hipSuccess;
        if (ok) ok = launch_batch(sl.d_jobs, m, sl.bs, 0, 0, sl.stream, &ex) == hipSuccess;
    }
    for (uint64_t id : ids) {
        SJob &j = s->jobs[id];
        if (!ok) j.status = DQMC_EDEVICE;
        if (j.status == DQMC_OK)
            (void)hipMemcpyAsync(j.h_count, j.d_count, 8, hipMemcpyDeviceToHost, sl.stream);
    }
    (void)hipEventRecord(sl.ev, sl.stream);
}

void retire(dqmc_server *s, Slot &sl)
{
    const double t = now_s();
    for (uint64_t id : sl.jobs) {
        SJob &j = s->jobs[id];
        j.count = *j.h_count;
        j.t_done = t;
        j.phase = kDone;
    }
    sl.jobs.clear();
    sl.busy = false;
}

void scheduler(dqmc_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool any_running = false, retired = false;
        for (auto *pool : {&s->big, &s->small})
            for (Slot &sl : *pool) {
                if (!sl.busy) continue;
                const hipError_t q = hipEventQuery(sl.ev);
                if (q == hipSuccess) {
                    retire(s, sl);
                    retired = true;
                } else if (q == hipErrorNotReady) {
                    any_running = true;
                } else {
                    // the slot's work failed: its jobs finish with an error
                    // instead of waiting forever
                    for (uint64_t id : sl.jobs) s->jobs[id].status = DQMC_EDEVICE;
                    retire(s, sl);
                    retired = true;
                }
            }
        if (retired) s->cv_done.notify_all();
        // on destruction: let running work finish, admit nothing more (a
        // queued job may wait for results that nobody will release)
        if (s->stop) {
            if (!any_running) break;
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
            continue;
        }
        // admission, first fit in arrival order (with aging of the head)
        std::vector<uint64_t> small_ids;
        Slot *free_small = nullptr;
        for (Slot &sl : s->small)
            if (!sl.busy) {
                free_small = &sl;
                break;
            }
        if (!s->queue.empty()) {
            if (s->queue.front() != s->head_id) {
                s->head_id = s->queue.front();
                s->head_since = now_s();
            }
        }
        for (auto it = s->queue.begin(); it != s->queue.end();) {
            SJob &j = s->jobs[*it];
            const bool is_head = it == s->queue.begin();
            const bool small = j.n <= kBatchMaxN;
            Slot *slot = nullptr;
            if (small) {
                if (free_small && small_ids.size() < kBatchSlotJobs) slot = free_small;
            } else {
                for (Slot &sl : s->big)
                    if (!sl.busy) {
                        slot = &sl;
                        break;
                    }
            }
            // small jobs from the top of the arena, large ones from the bottom
            if (slot != nullptr && !s->arena.alloc(j.fp, small, &j.off)) slot = nullptr;
            if (slot == nullptr) {
                if (is_head && now_s() - s->head_since > kAgingSeconds) break;  // let the head go first
                ++it;
                continue;
            }
            s->used += j.fp;
            j.phase = kRunning;
            j.t_admit = now_s();
            if (small) {
                small_ids.push_back(j.id);
            } else {
                launch_big(s, *slot, j);
                any_running = true;
            }
            it = s->queue.erase(it);
        }
        if (!small_ids.empty()) {
            launch_small(s, *free_small, small_ids);
            any_running = true;
        }
        // nothing runs and the queue cannot move: only released results can
        // free memory, so waiters are told instead of blocking forever
        const bool stalled = !any_running && !s->queue.empty();
        if (stalled != s->stalled) {
            s->stalled = stalled;
            if (stalled) s->cv_done.notify_all();
        }
        if (any_running)
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
}

}  // namespace

extern "C" {

int dqmc_server_create(int device, uint64_t budget_bytes, int32_t slots, dqmc_server **out)
{
    if (out == nullptr || slots < 0) return DQMC_EINVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return DQMC_EDEVICE;
    dqmc_server *s = new dqmc_server();
    s->device = device;
    if (slots == 0) slots = 4;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete s;
        return DQMC_EDEVICE;
    }
    bool ok = true;
    s->big.resize(slots);
    s->small.resize(2);
    for (auto *p : {&s->big, &s->small})
        for (Slot &sl : *p) {
            ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess;
            ok = ok && dqmc_create(device, &sl.ctx) == DQMC_OK;
        }
    for (Slot &sl : s->small) {
        ok = ok && hipHostMalloc((void **)&sl.h_jobs, kBatchSlotJobs * sizeof(dqmc_job), 0) == hipSuccess;
        ok = ok && hipMalloc((void **)&sl.d_jobs, kBatchSlotJobs * sizeof(dqmc_job)) == hipSuccess;
        ok = ok && hipMalloc(&sl.d_scratch, batch_scratch_bytes(kBatchSlotJobs)) == hipSuccess;
        if (ok) sl.bs = batch_scratch_at(sl.d_scratch, kBatchSlotJobs);
    }
    if (!ok) {
        dqmc_server_destroy(s);
        return DQMC_ENOMEM;
    }
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && budget_bytes == 0) budget_bytes = (uint64_t)(0.9 * (double)fr);
    budget_bytes &= ~uint64_t(255);
    if (budget_bytes == 0 || hipMalloc((void **)&s->arena_base, budget_bytes) != hipSuccess) {
        s->arena_base = nullptr;
        dqmc_server_destroy(s);
        return DQMC_ENOMEM;
    }
    s->arena.init(budget_bytes);
    s->budget = budget_bytes;
    s->thr = std::thread(scheduler, s);
    *out = s;
    return DQMC_OK;
}

int dqmc_server_submit(dqmc_server *s, int32_t n, const uint32_t *h_tt, uint64_t *id)
{
    if (s == nullptr || h_tt == nullptr || id == nullptr || n < 0 || n > DQMC_MAX_N) return DQMC_EINVAL;
    const uint64_t fp = footprint(n);
    if (fp > s->budget) return DQMC_ENOMEM;
    const uint64_t nw = tt_words_of(n);
    SJob j;
    j.n = n;
    j.fp = fp;
    if (hipHostMalloc((void **)&j.h_tt, nw * 4, 0) != hipSuccess ||
        hipHostMalloc((void **)&j.h_count, 8, 0) != hipSuccess) {
        if (j.h_tt) (void)hipHostFree(j.h_tt);
        return DQMC_ENOMEM;
    }
    memcpy(j.h_tt, h_tt, nw * 4);
    *j.h_count = 0;
    j.t_submit = now_s();
    {
        std::lock_guard<std::mutex> g(s->mu);
        j.id = s->next_id++;
        *id = j.id;
        s->jobs.emplace(j.id, j);
        s->queue.push_back(j.id);
    }
    s->cv_work.notify_one();
    return DQMC_OK;
}

static void fill_result(const SJob &j, dqmc_result *out)
{
    out->n = j.n;
    out->status = j.status;
    out->count = j.count;
    out->listed = j.count < j.cap ? j.count : j.cap;
    out->state = j.d_state;
    out->list = j.d_list;
    out->t_submit = j.t_submit;
    out->t_admit = j.t_admit;
    out->t_done = j.t_done;
}

int dqmc_server_poll(dqmc_server *s, uint64_t id, dqmc_result *out)
{
    if (s == nullptr) return DQMC_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end() || it->second.phase == kReleased) return DQMC_EINVAL;
    if (it->second.phase != kDone) return 0;
    if (out) fill_result(it->second, out);
    return 1;
}

int dqmc_server_wait(dqmc_server *s, uint64_t id, dqmc_result *out)
{
    if (s == nullptr) return DQMC_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end() || it->second.phase == kReleased) return DQMC_EINVAL;
    s->cv_done.wait(lk, [&] { return it->second.phase == kDone || (s->stalled && it->second.phase == kPending); });
    if (it->second.phase != kDone) {
        snprintf(s->err, sizeof(s->err), "job %llu cannot be admitted until results are released",
                 (unsigned long long)id);
        return DQMC_ENOMEM;
    }
    if (out) fill_result(it->second, out);
    return DQMC_OK;
}

int64_t dqmc_server_read(dqmc_server *s, uint64_t id, uint64_t *h_list, uint64_t cap)
{
    if (s == nullptr || (h_list == nullptr && cap > 0)) return DQMC_EINVAL;
    const uint64_t *src = nullptr;
    uint64_t k = 0;
    {
        // the scheduler needs the lock every round: hold it only to look the
        // job up, not during the copy
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->jobs.find(id);
        if (it == s->jobs.end() || it->second.phase != kDone) return DQMC_EINVAL;
        const SJob &j = it->second;
        k = j.count < j.cap ? j.count : j.cap;
        if (k > cap) k = cap;
        src = j.d_list;
    }
    if (k > 0 && hipMemcpy(h_list, src, k * 8, hipMemcpyDeviceToHost) != hipSuccess) return DQMC_EDEVICE;
    return (int64_t)k;
}

int dqmc_server_release(dqmc_server *s, uint64_t id)
{
    if (s == nullptr) return DQMC_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end() || it->second.phase != kDone) return DQMC_EINVAL;
    SJob &j = it->second;
    free_job_device(s, j);
    if (j.h_tt) (void)hipHostFree(j.h_tt);
    if (j.h_count) (void)hipHostFree(j.h_count);
    s->used -= j.fp;
    s->jobs.erase(it);
    s->stalled = false;
    s->cv_work.notify_one();
    return DQMC_OK;
}

void dqmc_server_destroy(dqmc_server *s)
{
    if (s == nullptr) return;
    if (s->thr.joinable()) {
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_one();
        s->thr.join();
    }
    (void)hipSetDevice(s->device);
    for (auto &kv : s->jobs) {
        free_job_device(s, kv.second);
        if (kv.second.h_tt) (void)hipHostFree(kv.second.h_tt);
        if (kv.second.h_count) (void)hipHostFree(kv.second.h_count);
    }
    for (auto *p : {&s->big, &s->small})
        for (Slot &sl : *p) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            if (sl.ctx) dqmc_destroy(sl.ctx);
            if (sl.ev) (void)hipEventDestroy(sl.ev);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
            if (sl.d_jobs) (void)hipFree(sl.d_jobs);
            if (sl.d_scratch) (void)hipFree(sl.d_scratch);
        }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

}  // extern "C"
