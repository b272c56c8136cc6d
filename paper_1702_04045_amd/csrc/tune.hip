// Autotuner of the z-plane stage (gfx950).
//
// Per plan and precision two launch choices of the plane kernel are free:
// the line schedule (threads per line and radix order of the n2 / n1
// transforms, PlaneSched) and the bands one work-group takes through its
// z-plane.  The bands per work-group only change how the work is dealt to
// work-groups, so results are bitwise the same for every choice; another
// schedule changes the rounding of the transforms (their radix order), not
// what they compute.  paro_plan_autotune times every candidate on the
// plan's own shape and keeps the fastest; the choice of a shape is kept for
// the process, so plans of the same shape tune once.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "paro_internal.h"

using namespace paro;

namespace {

constexpr int kBandChoices[] = {2, 4, 8, 16};
constexpr int kRowMapMax = 96;

struct RowMap {
    int32_t m[kRowMapMax];
};

// out[r n + p] = in[r n + map[p]]: every row of the plane potential moved
// from one schedule's thread order to another's
template <class VT> __global__ void k_relayout_rows(const VT *__restrict__ in, VT *__restrict__ out, RowMap map, int n,
                                                    int64_t total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t r = i / n;
    const int p = (int)(i - r * n);
    out[i] = in[r * n + map.m[p]];
}

template <class VT> int32_t relayout(const Plan &pl, VT *table, const RowMap &map)
{
    const int n = pl.grid[0];
    const int64_t total = (int64_t)pl.grid[0] * pl.grid[1] * pl.grid[2];
    VT *tmp = nullptr;
    PARO_HIP_TRY(hipMalloc(&tmp, sizeof(VT) * total));
    hipLaunchKernelGGL(k_relayout_rows<VT>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, pl.stream, table,
                       tmp, map, n, total);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(table, tmp, sizeof(VT) * total, hipMemcpyDeviceToDevice, pl.stream);
    const hipError_t es = hipStreamSynchronize(pl.stream);
    (void)hipFree(tmp);
    PARO_HIP_TRY(e);
    PARO_HIP_TRY(es);
    return PARO_OK;
}

int prec_slot(int32_t precision)
{
    switch (precision) {
    case PARO_PREC_FP64: return 0;
    case PARO_PREC_MIXED:
    case PARO_PREC_MIXED_BF16: return 1;
    default: return -1;
    }
}

bool bands_ok(int b) { return b >= 1 && b <= kPlaneBandsMax; }

// Select schedule `sched` and `bands` per work-group for precision slot pi,
// re-laying the potential table when the schedule changes.
int32_t select(Plan &pl, int pi, int sched, int bands)
{
    const int n = pl.grid[0];
    if (sched < 0 || sched >= plane_schedules(n) || !bands_ok(bands)) {
        set_error("paro_plan_set_schedule: schedule or bands out of range");
        return PARO_EINVAL;
    }
    if (sched != pl.plane_sched[pi]) {
        RowMap map{};
        if (n > kRowMapMax || !plane_row_map(n, pi == 1, pl.plane_sched[pi], sched, map.m)) {
            set_error("paro_plan_set_schedule: no row map between the schedules");
            return PARO_EINVAL;
        }
        const int32_t rc = pi == 0 ? relayout(pl, pl.vplane, map) : relayout(pl, pl.vplane32, map);
        if (rc) return rc;
    }
    pl.plane_sched[pi] = sched;
    pl.plane_bands[pi] = bands;
    return PARO_OK;
}

// milliseconds of one plane stage over nb bands with the plan's current
// choice: best of three runs of `reps` stages
int32_t time_plane(const Plan &pl, const Workspace &w, int nb, bool fp32, hipEvent_t e0, hipEvent_t e1, int reps,
                   double *ms)
{
    double best = 1e300;
    for (int trial = 0; trial < 3; ++trial) {
        PARO_HIP_TRY(hipEventRecord(e0, pl.stream));
        for (int r = 0; r < reps; ++r) PARO_HIP_TRY(launch_plane_only(pl, w, nb, fp32));
        PARO_HIP_TRY(hipEventRecord(e1, pl.stream));
        PARO_HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        PARO_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        best = std::min(best, (double)t / reps);
    }
    *ms = best;
    return PARO_OK;
}

struct Choice {
    int sched, bands;
    double ms, ms_default;
    int candidates;
};
using ShapeKey = std::tuple<int, int, int, int, int, int, int>;  // grid, nst, ncol, nmax1, nb, slot
std::mutex g_mu;
std::map<ShapeKey, Choice> g_choices;

struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

int32_t tune_slot(Plan &pl, const Workspace &w, int nb, int pi, Events &ev, Choice *out)
{
    const int n = pl.grid[0];
    const int cbmax = std::min(nb, pi == 1 ? kMaxBandsPerChunk32 : kMaxBandsPerChunk);
    const int sched0 = pl.plane_sched[pi], bands0 = pl.plane_bands[pi];
    int32_t dsched = 0, dbands = kPlaneBandsDefault;  // a new plan's choice
    plane_default(n, pi, &dsched, &dbands);
    Choice best{dsched, dbands, 1e300, 0.0, 0};
    // one untimed stage, then the repetitions that make about a millisecond
    pl.plane_sched[pi] = dsched;
    pl.plane_bands[pi] = dbands;
    PARO_HIP_TRY(launch_plane_only(pl, w, nb, pi == 1));
    double t1 = 0.0;
    int32_t rc = time_plane(pl, w, nb, pi == 1, ev.e0, ev.e1, 1, &t1);
    if (rc) return rc;
    const int reps = std::max(2, std::min(64, (int)(1.0 / std::max(t1, 1e-3)) + 1));
    for (int v = 0; v < plane_schedules(n); ++v) {
        int prev = 0;
        for (int b : kBandChoices) {
            if (prev >= cbmax) break;  // one work-group per plane already covers every band
            prev = b;
            pl.plane_sched[pi] = v;
            pl.plane_bands[pi] = b;
            PARO_HIP_TRY(launch_plane_only(pl, w, nb, pi == 1));
            double ms = 0.0;
            rc = time_plane(pl, w, nb, pi == 1, ev.e0, ev.e1, reps, &ms);
            if (rc) return rc;
            ++best.candidates;
            if (v == dsched && b == dbands) best.ms_default = ms;
            if (ms < best.ms) {
                best.sched = v;
                best.bands = b;
                best.ms = ms;
            }
        }
    }
    // keep the default unless a candidate is more than 1 % faster
    if (best.ms_default > 0.0 && best.ms_default <= 1.01 * best.ms) {
        best.sched = dsched;
        best.bands = dbands;
        best.ms = best.ms_default;
    }
    pl.plane_sched[pi] = sched0;
    pl.plane_bands[pi] = bands0;
    *out = best;
    return PARO_OK;
}

}  // namespace

extern "C" {

int32_t paro_plan_set_schedule(paro_plan plan, int32_t precision, int32_t schedule, int32_t bands)
{
    const int pi = prec_slot(precision);
    if (!plan || pi < 0) {
        set_error("paro_plan_set_schedule: bad argument");
        return PARO_EINVAL;
    }
    return select(plan->pl, pi, schedule, bands);
}

int32_t paro_plan_get_schedule(paro_plan plan, int32_t precision, int32_t *schedule, int32_t *bands,
                               int32_t *n_schedules)
{
    const int pi = prec_slot(precision);
    if (!plan || pi < 0) {
        set_error("paro_plan_get_schedule: bad argument");
        return PARO_EINVAL;
    }
    if (schedule) *schedule = plan->pl.plane_sched[pi];
    if (bands) *bands = plan->pl.plane_bands[pi];
    if (n_schedules) *n_schedules = plane_schedules(plan->pl.grid[0]);
    return PARO_OK;
}

int32_t paro_plan_autotune(paro_plan plan, int32_t nb, void *ws, size_t ws_bytes, int32_t flags,
                           paro_tune_result *result)
{
    if (!plan || nb <= 0 || nb > 1024 || !ws || (flags & ~PARO_TUNE_FORCE)) {
        set_error("paro_plan_autotune: bad argument");
        return PARO_EINVAL;
    }
    Plan &pl = plan->pl;
    if (reinterpret_cast<uintptr_t>(ws) % 256) {
        set_error("workspace must be 256-byte aligned");
        return PARO_EINVAL;
    }
    if (ws_bytes < workspace_bytes(pl, nb)) {
        set_error("workspace smaller than paro_workspace_bytes");
        return PARO_ESIZE;
    }
    paro_tune_result res;
    std::memset(&res, 0, sizeof(res));
    if (big_grid(pl.grid[0])) {
        // one plane kernel and one launch shape above 96 points: nothing to choose
        for (int pi = 0; pi < 2; ++pi) {
            res.schedule[pi] = pl.plane_sched[pi];
            res.bands[pi] = pl.plane_bands[pi];
        }
        if (result) *result = res;
        return PARO_OK;
    }
    const Workspace w = carve_workspace(pl, nb, ws);
    const size_t stick_bytes =
        std::max(sizeof(double2) * (size_t)std::min(nb, kMaxBandsPerChunk),
                 sizeof(float2) * (size_t)std::min(nb, kMaxBandsPerChunk32)) *
        (size_t)pl.grid[2] * (size_t)pl.nst;
    PARO_HIP_TRY(hipMemsetAsync(w.sticks, 0, stick_bytes, pl.stream));
    Events ev;
    PARO_HIP_TRY(hipEventCreate(&ev.e0));
    PARO_HIP_TRY(hipEventCreate(&ev.e1));
    res.cached = 1;
    for (int pi = 0; pi < 2; ++pi) {
        const ShapeKey key{pl.grid[0], pl.nst, pl.ncol, pl.nmax[0], nb, pi, pl.grid[2]};
        Choice c{};
        bool have = false;
        if (!(flags & PARO_TUNE_FORCE)) {
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = g_choices.find(key);
            if (it != g_choices.end()) {
                c = it->second;
                have = true;
            }
        }
        if (!have) {
            res.cached = 0;
            const int32_t rc = tune_slot(pl, w, nb, pi, ev, &c);
            if (rc) return rc;
            std::lock_guard<std::mutex> lk(g_mu);
            g_choices[key] = c;
        }
        const int32_t rc = select(pl, pi, c.sched, c.bands);
        if (rc) return rc;
        res.schedule[pi] = c.sched;
        res.bands[pi] = c.bands;
        res.ms[pi] = c.ms;
        res.ms_default[pi] = c.ms_default;
        res.candidates = c.candidates;
    }
    PARO_HIP_TRY(hipStreamSynchronize(pl.stream));
    if (result) *result = res;
    return PARO_OK;
}

}  // extern "C"
