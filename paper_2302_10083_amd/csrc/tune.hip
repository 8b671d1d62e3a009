// Autotuning of the launch choices that leave results unchanged: the
// column-pass occupancy cap and item order of a batch plan, and the digit-group plan of
// the single-function pipeline.  Candidates are timed on the caller's own
// buffers with HIP events on the caller's stream; the fastest is applied
// through the public configuration calls (dqmc_batch_config, dqmc_set_plan).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "api_types.h"
#include "dqmc.h"
#include "launch.h"

using dqmc::kMaxGroupStart;

namespace {

constexpr int kLowDigits = 12;
constexpr int kMaxGroup = 6;

int tune_fail(dqmc_ctx *ctx, int code, const char *msg)
{
    if (ctx) snprintf(ctx->err, sizeof(ctx->err), "%s", msg);
    return code;
}

// Times `reps` runs of f on stream s after one untimed run; returns the
// fastest run in milliseconds, or a negative value on a HIP error or a
// failing run (its status in *rc).
template <typename F>
float time_best(hipStream_t s, int reps, int *rc, F &&f)
{
    *rc = f();
    if (*rc != DQMC_OK) return -1.0f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0f;
    }
    float best = -1.0f;
    for (int r = 0; r < reps; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) break;
        *rc = f();
        if (*rc != DQMC_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            best = -1.0f;
            break;
        }
        if (best < 0.0f || ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return *rc == DQMC_OK ? best : -1.0f;
}

// Every ordered split of h digits into k groups of 1..kMaxGroup digits, in
// lexicographic order of the sizes.
void splits(int h, int k, std::vector<int> &cur, std::vector<std::vector<int>> &out, size_t limit)
{
    if (out.size() >= limit) return;
    if (k == 0) {
        if (h == 0) out.push_back(cur);
        return;
    }
    for (int s = 1; s <= kMaxGroup && s <= h; ++s) {
        if (h - s > (k - 1) * kMaxGroup) continue;  // the rest cannot fit
        cur.push_back(s);
        splits(h - s, k - 1, cur, out, limit);
        cur.pop_back();
    }
}

// Reader of the tuning file's JSON subset: objects, arrays, strings (escapes
// \\ and \" only) and integers.
struct JsonReader {
    const char *p, *end;
    bool ok = true;

    void ws()
    {
        while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
    }
    bool peek(char c)
    {
        ws();
        return p < end && *p == c;
    }
    bool take(char c)
    {
        if (!peek(c)) return ok = false;
        ++p;
        return true;
    }
    bool str(std::string &out)
    {
        out.clear();
        if (!take('"')) return false;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                if (++p >= end || (*p != '"' && *p != '\\')) return ok = false;
            }
            out.push_back(*p++);
        }
        if (p >= end) return ok = false;
        ++p;
        return true;
    }
    bool integer(long &v)
    {
        ws();
        const char *q = p;
        bool neg = false;
        if (q < end && *q == '-') {
            neg = true;
            ++q;
        }
        if (q >= end || *q < '0' || *q > '9') return ok = false;
        long x = 0;
        while (q < end && *q >= '0' && *q <= '9') {
            x = x * 10 + (*q++ - '0');
            if (x > 1000000) return ok = false;
        }
        p = q;
        v = neg ? -x : x;
        return true;
    }
    // key-value pairs of an object: f(key) reads the value, false on error
    template <typename F>
    bool object(F &&f)
    {
        if (!take('{')) return false;
        if (peek('}')) return take('}');
        std::string key;
        do {
            if (!str(key) || !take(':') || !f(key)) return ok = false;
        } while (peek(',') && take(','));
        return take('}');
    }
    template <typename F>
    bool array(F &&f)
    {
        if (!take('[')) return false;
        if (peek(']')) return take(']');
        do {
            if (!f()) return ok = false;
        } while (peek(',') && take(','));
        return take(']');
    }
};

struct TuneEntry {
    long n = -1, split = -1;
    std::vector<int32_t> groups;
};

int device_arch(const dqmc_ctx *ctx, std::string &arch)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return DQMC_EDEVICE;
    arch = prop.gcnArchName;
    return DQMC_OK;
}

}  // namespace

extern "C" {

int dqmc_batch_autotune(dqmc_batch *plan, int32_t reps, void *stream, dqmc_batch_trial *trials, int32_t cap_trials,
                        int32_t *ntrials)
{
    if (ntrials != nullptr) *ntrials = 0;
    if (plan == nullptr || reps < 1 || cap_trials < 0 || (trials == nullptr && cap_trials > 0)) return DQMC_EINVAL;
    dqmc_ctx *ctx = plan->ctx;
    ctx->err[0] = 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return tune_fail(ctx, DQMC_EDEVICE, "hipSetDevice failed");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return tune_fail(ctx, DQMC_EINVAL, "autotuning cannot run while the stream is captured");
    const int caps[] = {0, 1, 2, 3};  // column-pass workgroups per CU (0: as many as the registers allow, 4)
    int32_t best_cap = plan->col_cap, best_order = plan->order_mode, n = 0;
    float best = -1.0f;
    for (int order = 0; order < dqmc::kBatchModes; ++order) {
        for (int cap : caps) {
            int rc = dqmc_batch_config(plan, cap, order);
            if (rc != DQMC_OK) return rc;
            const float ms = time_best((hipStream_t)stream, reps, &rc, [&] { return dqmc_batch_run(plan, stream); });
            if (rc != DQMC_OK) return rc;
            if (ms < 0.0f) return tune_fail(ctx, DQMC_EDEVICE, "timing a batch candidate failed");
            if (n < cap_trials) trials[n] = dqmc_batch_trial{cap, order, ms};
            ++n;
            if (best < 0.0f || ms < best) {
                best = ms;
                best_cap = cap;
                best_order = order;
            }
        }
    }
    if (ntrials != nullptr) *ntrials = n;
    return dqmc_batch_config(plan, best_cap, best_order);
}

int dqmc_plan_autotune(dqmc_ctx *ctx, int n, const uint32_t *d_tt, uint32_t *d_state, uint64_t *d_count,
                       int32_t extra_groups, int32_t reps, void *stream, dqmc_plan_trial *trials, int32_t cap,
                       int32_t *ntrials)
{
    if (ntrials != nullptr) *ntrials = 0;
    if (ctx == nullptr) return DQMC_EINVAL;
    ctx->err[0] = 0;
    if (n <= kLowDigits || n > DQMC_MAX_N) return tune_fail(ctx, DQMC_EINVAL, "plan tuning needs 12 < n <= 25");
    if (extra_groups < 0 || extra_groups > 2 || reps < 1 || cap < 0 || (trials == nullptr && cap > 0))
        return tune_fail(ctx, DQMC_EINVAL, "bad extra_groups, reps or trial buffer");
    if (d_tt == nullptr || d_state == nullptr || d_count == nullptr)
        return tune_fail(ctx, DQMC_EINVAL, "NULL truth table, state or count");
    if (hipSetDevice(ctx->device) != hipSuccess) return tune_fail(ctx, DQMC_EDEVICE, "hipSetDevice failed");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return tune_fail(ctx, DQMC_EINVAL, "autotuning cannot run while the stream is captured");
    const int h = n - kLowDigits, kmin = (h + kMaxGroup - 1) / kMaxGroup;
    std::vector<std::vector<int>> cands;
    std::vector<int> cur;
    for (int k = kmin; k <= std::min(h, kmin + extra_groups); ++k) splits(h, k, cur, cands, DQMC_MAX_PLAN_TRIALS);
    // plans whose top group starts above digit kMaxGroupStart are not valid
    // (dqmc_set_plan rejects them)
    cands.erase(std::remove_if(cands.begin(), cands.end(),
                               [&](const std::vector<int> &c) { return n - c.back() + 1 > kMaxGroupStart; }),
                cands.end());
    // the plan and split mode in force are restored if a run fails
    int32_t keep[DQMC_MAX_N];
    const int nkeep = ctx->plan_len[n], keep_split = ctx->split[n];
    for (int i = 0; i < nkeep; ++i) keep[i] = ctx->plan[n][i];
    auto restore = [&](int rc) {
        (void)dqmc_set_plan(ctx, n, keep, nkeep);
        ctx->split[n] = keep_split;
        return rc;
    };
    ctx->split[n] = 0;  // the group plans are timed on the whole-state passes
    int best_i = -1, count = 0;
    float best = -1.0f;
    for (size_t i = 0; i < cands.size(); ++i) {
        std::vector<int32_t> sz(cands[i].begin(), cands[i].end());
        int rc = dqmc_set_plan(ctx, n, sz.data(), (int)sz.size());
        if (rc != DQMC_OK) return restore(rc);
        const float ms = time_best((hipStream_t)stream, reps, &rc,
                                   [&] { return dqmc_primes(ctx, n, d_tt, d_state, nullptr, 0, d_count, stream); });
        if (rc != DQMC_OK) return restore(rc);
        if (ms < 0.0f) return restore(tune_fail(ctx, DQMC_EDEVICE, "timing a plan candidate failed"));
        if (count < cap) {
            dqmc_plan_trial &t = trials[count];
            t.ngroups = (int32_t)sz.size();
            for (int g = 0; g < DQMC_MAX_N; ++g) t.sizes[g] = g < (int)sz.size() ? sz[g] : 0;
            t.ms = ms;
        }
        ++count;
        if (best < 0.0f || ms < best) {
            best = ms;
            best_i = (int)i;
        }
    }
    // the top-digit split (three (n-1)-variable slices) as one more candidate
    ctx->split[n] = 1;
    int rc = DQMC_OK;
    const float ms_split = time_best((hipStream_t)stream, reps, &rc,
                                     [&] { return dqmc_primes(ctx, n, d_tt, d_state, nullptr, 0, d_count, stream); });
    if (rc != DQMC_OK) return restore(rc);
    if (ms_split < 0.0f) return restore(tune_fail(ctx, DQMC_EDEVICE, "timing the split candidate failed"));
    if (count < cap) {
        dqmc_plan_trial &t = trials[count];
        t.ngroups = 0;
        for (int g = 0; g < DQMC_MAX_N; ++g) t.sizes[g] = 0;
        t.ms = ms_split;
    }
    ++count;
    if (ntrials != nullptr) *ntrials = count;
    ctx->split[n] = ms_split < best ? 1 : 0;
    std::vector<int32_t> win(cands[best_i].begin(), cands[best_i].end());
    return dqmc_set_plan(ctx, n, win.data(), (int)win.size());
}

int dqmc_tune_save(const dqmc_ctx *ctx, const char *path)
{
    if (ctx == nullptr || path == nullptr) return DQMC_EINVAL;
    std::string arch;
    if (device_arch(ctx, arch) != DQMC_OK) return DQMC_EDEVICE;
    std::string out = "{\"format\": \"dqmc-tune-1\", \"arch\": \"";
    for (char c : arch) {
        if (c == '"' || c == '\\') out.push_back('\\');
        out.push_back(c);
    }
    out += "\",\n \"plans\": [";
    bool first = true;
    for (int n = kLowDigits + 1; n <= DQMC_MAX_N; ++n) {
        if (ctx->plan_len[n] == 0 && ctx->split[n] < 0) continue;
        char buf[64];
        snprintf(buf, sizeof(buf), "%s\n  {\"n\": %d, \"groups\": [", first ? "" : ",", n);
        out += buf;
        for (int g = 0; g < ctx->plan_len[n]; ++g) {
            snprintf(buf, sizeof(buf), "%s%d", g ? ", " : "", ctx->plan[n][g]);
            out += buf;
        }
        snprintf(buf, sizeof(buf), "], \"split\": %d}", ctx->split[n]);
        out += buf;
        first = false;
    }
    out += "]}\n";
    FILE *f = fopen(path, "wb");
    if (f == nullptr) return DQMC_EIO;
    const bool ok = fwrite(out.data(), 1, out.size(), f) == out.size();
    return (fclose(f) == 0 && ok) ? DQMC_OK : DQMC_EIO;
}

int dqmc_tune_load(dqmc_ctx *ctx, const char *path, int32_t *napplied)
{
    if (ctx == nullptr || path == nullptr) return DQMC_EINVAL;
    if (napplied != nullptr) *napplied = 0;
    FILE *f = fopen(path, "rb");
    if (f == nullptr) return tune_fail(ctx, DQMC_EIO, "cannot open the tuning file");
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) {
        text.append(buf, got);
        if (text.size() > (1u << 20)) break;
    }
    const bool read_ok = !ferror(f) && text.size() <= (1u << 20);
    fclose(f);
    if (!read_ok) return tune_fail(ctx, DQMC_EIO, "cannot read the tuning file");
    JsonReader r{text.data(), text.data() + text.size()};
    std::string format, arch;
    std::vector<TuneEntry> entries;
    r.object([&](const std::string &key) {
        if (key == "format") return r.str(format);
        if (key == "arch") return r.str(arch);
        if (key != "plans") return false;
        return r.array([&] {
            TuneEntry e;
            const bool ok = r.object([&](const std::string &k) {
                if (k == "n") return r.integer(e.n);
                if (k == "split") return r.integer(e.split);
                if (k != "groups") return false;
                return r.array([&] {
                    long g;
                    if (!r.integer(g)) return false;
                    e.groups.push_back((int32_t)g);
                    return e.groups.size() <= (size_t)DQMC_MAX_N;
                });
            });
            entries.push_back(e);
            return ok;
        });
    });
    r.ws();
    if (!r.ok || r.p != r.end || format != "dqmc-tune-1")
        return tune_fail(ctx, DQMC_EINVAL, "malformed tuning file");
    std::string mine;
    if (device_arch(ctx, mine) != DQMC_OK) return tune_fail(ctx, DQMC_EDEVICE, "cannot read the device properties");
    if (arch != mine) return DQMC_OK;  // written for another architecture
    // apply all or nothing
    int plan_len[DQMC_MAX_N + 1], split[DQMC_MAX_N + 1], plan[DQMC_MAX_N + 1][DQMC_MAX_N];
    memcpy(plan_len, ctx->plan_len, sizeof(plan_len));
    memcpy(split, ctx->split, sizeof(split));
    memcpy(plan, ctx->plan, sizeof(plan));
    int rc = DQMC_OK;
    for (const TuneEntry &e : entries) {
        if (e.n <= kLowDigits || e.n > DQMC_MAX_N) {
            rc = tune_fail(ctx, DQMC_EINVAL, "tuning entry with n outside 13..25");
            break;
        }
        rc = dqmc_set_plan(ctx, (int)e.n, e.groups.data(), (int)e.groups.size());
        if (rc == DQMC_OK) rc = dqmc_set_split(ctx, (int)e.n, (int)e.split);
        if (rc != DQMC_OK) break;
    }
    if (rc != DQMC_OK) {
        memcpy(ctx->plan_len, plan_len, sizeof(plan_len));
        memcpy(ctx->split, split, sizeof(split));
        memcpy(ctx->plan, plan, sizeof(plan));
        return rc;
    }
    if (napplied != nullptr) *napplied = (int32_t)entries.size();
    return DQMC_OK;
}

}  // extern "C"
