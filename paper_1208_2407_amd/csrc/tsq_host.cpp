// C ABI of the second-order Trotter-Suzuki solver: validation, FP64
// coefficients, workspace layout, the pass schedule and kernel launches.
// The operations and their citations are documented in include/tsq.h.

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tsq.h"
#include "tsq_internal.h"

struct tsq_plan {
    tsq_problem p;
    double Jx, Jy, eps0;
    tsq::Coef64 oxh, oyh, ox2, oy2;
    tsq_schedule sched;   // resolved (segment_rows may stay 0 = per launch)
    size_t sites, elem, pelem;
    size_t off_psi2, off_ptab, off_scratch, ws_bytes;
    const void* ws_bound;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return TSQ_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Block exponential of hopping energy J acting for tau: s = sin al,
// d = 1 - cos al = 2 sin^2(al/2), al = tau J / hbar.
tsq::Coef64 block_coef(double tau, double J, double hbar) {
    const double al = tau * J / hbar;
    const double h = std::sin(0.5 * al);
    return tsq::Coef64{std::sin(al), 2.0 * h * h};
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

constexpr size_t kScratchBytes = (2 * tsq::kReduceBlocks + 2) * sizeof(double);

// Default schedule.  Steps per pass: 4 (the deepest fusion built).  Segment
// height: as many wavefront tiles as the device holds resident at once (one
// round, no tail of a partly filled second round), each segment at least 2K
// row pairs long so the discarded warm-up pairs stay below half the work.
constexpr int kDefaultSteps = 4;

// Fill the zero fields of a requested schedule with defaults; false if the
// combination has no kernel instance.
bool resolve_schedule(const tsq_schedule& in, tsq_schedule& out) {
    out = in;
    if (out.steps_per_pass == 0) out.steps_per_pass = kDefaultSteps;
    if (out.phase_store == 0) out.phase_store = out.steps_per_pass <= tsq::kMaxRegSteps ? 1 : 2;
    if (out.pairs_per_lane == 0) out.pairs_per_lane = 1;
    if (out.phase_store == 1 && out.steps_per_pass > tsq::kMaxRegSteps) return false;
    if (out.phase_store == 2 && out.pairs_per_lane != 1) return false;
    return true;
}

struct DeviceShape {
    int device = -1;
    int cus = 0;
};
thread_local DeviceShape g_dev;

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (g_dev.device != dev) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
        g_dev.device = dev;
        g_dev.cus = cus;
    }
    return g_dev.cus;
}

int occupancy_cached(int dtype, int steps, bool last, int ppl, bool lds) {
    // [dtype][steps][last][ppl][lds]; 0 = not yet queried
    static std::atomic<int> table[2][tsq::kMaxSteps + 1][2][3][2];
    std::atomic<int>& slot = table[dtype & 1][steps][last ? 1 : 0][ppl][lds ? 1 : 0];
    int v = slot.load(std::memory_order_relaxed);
    if (v == 0) {
        v = tsq::march_blocks_per_cu(dtype, steps, last, ppl, lds);
        if (v <= 0) v = 1;
        slot.store(v, std::memory_order_relaxed);
    }
    return v;
}

int default_seg_rows(const tsq_plan* p, int steps, bool last, int ppl, bool lds) {
    const tsq::MarchGeometry g = tsq::march_geometry(p->p.nx, p->p.ny, steps, last, ppl, 2);
    int cus = device_cus();
    if (cus <= 0) cus = 256;
    const long long slots =
        (long long)cus * occupancy_cached(p->p.dtype, steps, last, ppl, lds) * tsq::kWavesPerBlock;
    const long long pairs = p->p.ny / 2;
    long long segs = slots / g.nstrips;
    if (segs < 1) segs = 1;
    if (segs > pairs) segs = pairs;
    long long pairs_per_seg = (pairs + segs - 1) / segs;
    const long long min_pairs = 2LL * (steps + (last ? 1 : 0));
    if (pairs_per_seg < min_pairs) pairs_per_seg = min_pairs;
    return (int)(2 * pairs_per_seg);
}

// Pass sizes as runs of (steps per pass, repeat): S steps each, the remainder
// in the last pass.  An odd pass count would leave the result in the second
// buffer, so the last pass holding more than one step is split in two; if no
// pass can be split the caller copies the result back.
struct Run {
    int size;
    int64_t count;
};

bool pass_runs(int64_t steps, int S, std::vector<Run>& runs) {
    runs.clear();
    const int64_t full = steps / S;
    const int rem = (int)(steps % S);
    if (full > 0) runs.push_back(Run{S, full});
    if (rem > 0) runs.push_back(Run{rem, 1});
    const int64_t total = full + (rem > 0 ? 1 : 0);
    if (!(total & 1)) return false;
    for (size_t i = runs.size(); i-- > 0;) {
        if (runs[i].size < 2) continue;
        const Run r = runs[i];
        const int a = r.size / 2, b = r.size - a;
        std::vector<Run> tail(runs.begin() + i + 1, runs.end());
        runs.resize(i);
        if (r.count > 1) runs.push_back(Run{r.size, r.count - 1});
        runs.push_back(Run{a, 1});
        runs.push_back(Run{b, 1});
        runs.insert(runs.end(), tail.begin(), tail.end());
        return false;
    }
    return true;
}

int64_t run_passes(const std::vector<Run>& runs) {
    int64_t n = 0;
    for (const Run& r : runs) n += r.count;
    return n;
}

int check_ws(const tsq_plan* plan, const void* ws, size_t ws_bytes) {
    if (ws == nullptr) return fail(TSQ_ERR_ARG, "workspace pointer is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(TSQ_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < plan->ws_bytes)
        return fail(TSQ_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                    ws_bytes, plan->ws_bytes);
    return TSQ_OK;
}

}  // namespace

extern "C" {

int tsq_abi_version(void) { return TSQ_ABI_VERSION; }

const char* tsq_last_error(void) { return g_err.c_str(); }

int tsq_plan_create(const tsq_problem* pr, tsq_plan** out) {
    if (pr == nullptr || out == nullptr) return fail(TSQ_ERR_ARG, "null problem or output pointer");
    if (pr->nx < 2 || pr->ny < 2)
        return fail(TSQ_ERR_SHAPE, "mesh %d x %d: each side must be >= 2", pr->nx, pr->ny);
    if (pr->bc != TSQ_BC_PERIODIC && pr->bc != TSQ_BC_CLOSED)
        return fail(TSQ_ERR_ARG, "unknown boundary condition %d", pr->bc);
    if (pr->bc == TSQ_BC_PERIODIC && ((pr->nx & 1) || (pr->ny & 1)))
        return fail(TSQ_ERR_SHAPE,
                    "mesh %d x %d: periodic boundaries need even sides (pairs must tile each line)",
                    pr->nx, pr->ny);
    if ((long long)pr->nx * (long long)pr->ny > 0x7fffffffLL)
        return fail(TSQ_ERR_SHAPE, "mesh %d x %d exceeds 2^31-1 sites", pr->nx, pr->ny);
    if (!finite_pos(pr->dx) || !finite_pos(pr->dy))
        return fail(TSQ_ERR_ARG, "spacings must be finite and > 0 (dx=%g, dy=%g)", pr->dx, pr->dy);
    if (!finite_pos(pr->mass)) return fail(TSQ_ERR_ARG, "mass must be finite and > 0 (%g)", pr->mass);
    if (!finite_pos(pr->hbar)) return fail(TSQ_ERR_ARG, "hbar must be finite and > 0 (%g)", pr->hbar);
    if (!std::isfinite(pr->dt)) return fail(TSQ_ERR_ARG, "dt must be finite (%g)", pr->dt);
    if (pr->dtype != TSQ_C64 && pr->dtype != TSQ_C128)
        return fail(TSQ_ERR_DTYPE, "unknown dtype %d", pr->dtype);
    if (pr->bc == TSQ_BC_CLOSED)
        return fail(TSQ_ERR_UNSUPPORTED, "closed boundaries are not implemented in this build");

    tsq_plan* p = new (std::nothrow) tsq_plan();
    if (!p) return fail(TSQ_ERR_ARG, "out of host memory");
    p->p = *pr;
    const double hb = pr->hbar, m = pr->mass;
    p->Jx = hb * hb / (2.0 * m * pr->dx * pr->dx);
    p->Jy = hb * hb / (2.0 * m * pr->dy * pr->dy);
    p->eps0 = hb * hb / (m * pr->dx * pr->dx) + hb * hb / (m * pr->dy * pr->dy);
    const double h = 0.5 * pr->dt;
    p->oxh = block_coef(h, p->Jx, hb);
    p->oyh = block_coef(h, p->Jy, hb);
    p->ox2 = block_coef(pr->dt, p->Jx, hb);
    p->oy2 = block_coef(pr->dt, p->Jy, hb);
    resolve_schedule(tsq_schedule{0, 0, 0, 0}, p->sched);
    p->sites = (size_t)pr->nx * (size_t)pr->ny;
    p->elem = pr->dtype == TSQ_C128 ? 16 : 8;
    p->pelem = 16;  // complex128: exp(-i phi); complex64: hi + lo complex floats
    p->off_psi2 = 0;
    p->off_ptab = align_up(p->sites * p->elem, 256);
    p->off_scratch = align_up(p->off_ptab + p->sites * p->pelem, 256);
    p->ws_bytes = p->off_scratch + kScratchBytes;
    p->ws_bound = nullptr;
    *out = p;
    return ok();
}

int tsq_plan_destroy(tsq_plan* plan) {
    delete plan;
    return ok();
}

int tsq_workspace_size(const tsq_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(TSQ_ERR_ARG, "null plan or output pointer");
    *bytes = plan->ws_bytes;
    return ok();
}

int tsq_plan_set_schedule(tsq_plan* plan, const tsq_schedule* sc) {
    if (!plan || !sc) return fail(TSQ_ERR_ARG, "null plan or schedule");
    if (sc->steps_per_pass < 0 || sc->steps_per_pass > tsq::kMaxSteps)
        return fail(TSQ_ERR_ARG, "steps_per_pass %d outside 0..%d", sc->steps_per_pass,
                    tsq::kMaxSteps);
    if (sc->segment_rows < 0 || (sc->segment_rows & 1))
        return fail(TSQ_ERR_ARG, "segment_rows %d must be even and >= 0", sc->segment_rows);
    if (sc->pairs_per_lane < 0 || sc->pairs_per_lane > 2)
        return fail(TSQ_ERR_ARG, "pairs_per_lane %d outside 0..2", sc->pairs_per_lane);
    if (sc->phase_store < 0 || sc->phase_store > 2)
        return fail(TSQ_ERR_ARG, "phase_store %d outside 0..2", sc->phase_store);
    tsq_schedule r;
    if (!resolve_schedule(*sc, r))
        return fail(TSQ_ERR_ARG,
                    "no kernel for steps_per_pass %d, pairs_per_lane %d, phase_store %d "
                    "(registers hold at most %d steps; LDS needs 1 pair per lane)",
                    r.steps_per_pass, r.pairs_per_lane, r.phase_store, tsq::kMaxRegSteps);
    plan->sched = r;
    return ok();
}

int tsq_plan_get_schedule(const tsq_plan* plan, tsq_schedule* sc) {
    if (!plan || !sc) return fail(TSQ_ERR_ARG, "null argument");
    *sc = plan->sched;
    return ok();
}

int tsq_evolve_passes(const tsq_plan* plan, int64_t steps, int64_t* passes, int32_t* copy_back) {
    if (!plan || !passes || !copy_back) return fail(TSQ_ERR_ARG, "null argument");
    if (steps < 0) return fail(TSQ_ERR_ARG, "steps must be >= 0 (%lld)", (long long)steps);
    std::vector<Run> runs;
    const bool cb = steps > 0 && pass_runs(steps, plan->sched.steps_per_pass, runs);
    *passes = run_passes(runs);
    *copy_back = cb ? 1 : 0;
    return ok();
}

int tsq_set_potential(tsq_plan* plan, const double* V, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !V) return fail(TSQ_ERR_ARG, "null plan or potential");
    int rc = check_ws(plan, ws, ws_bytes);
    if (rc) return rc;
    char* w = static_cast<char*>(ws);
    hipError_t e = tsq::launch_phase_table(plan->p.dtype, V, w + plan->off_ptab,
                                           (long long)plan->sites, plan->p.dt, plan->eps0,
                                           plan->p.hbar, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "phase table launch: %s", hipGetErrorString(e));
    plan->ws_bound = ws;
    return ok();
}

int tsq_evolve(tsq_plan* plan, void* psi, int64_t steps, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !psi) return fail(TSQ_ERR_ARG, "null plan or psi");
    if (steps < 0) return fail(TSQ_ERR_ARG, "steps must be >= 0 (%lld)", (long long)steps);
    if (reinterpret_cast<uintptr_t>(psi) % 16 != 0) return fail(TSQ_ERR_ARG, "psi must be 16-byte aligned");
    int rc = check_ws(plan, ws, ws_bytes);
    if (rc) return rc;
    if (plan->ws_bound == nullptr) return fail(TSQ_ERR_STATE, "tsq_set_potential has not been called");
    if (plan->ws_bound != ws)
        return fail(TSQ_ERR_STATE, "workspace differs from the one given to tsq_set_potential");
    if (steps == 0) return ok();

    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    void* buf[2] = {psi, w + plan->off_psi2};
    const int S = plan->sched.steps_per_pass;
    const int ppl = plan->sched.pairs_per_lane;
    const bool lds = plan->sched.phase_store == 2;

    std::vector<Run> runs;
    const bool copy_back = pass_runs(steps, S, runs);
    const int64_t npasses = run_passes(runs);

    tsq::PassDesc d;
    d.ptab = w + plan->off_ptab;
    d.nx = plan->p.nx;
    d.ny = plan->p.ny;
    d.pairs_per_lane = ppl;
    d.phase_lds = lds;
    d.oxh = plan->oxh;
    d.oyh = plan->oyh;
    d.ox2 = plan->ox2;
    d.oy2 = plan->oy2;
    int64_t i = 0;
    for (const Run& r : runs) {
        for (int64_t k = 0; k < r.count; ++k, ++i) {
            d.src = buf[i & 1];
            d.dst = buf[(i + 1) & 1];
            d.steps = r.size;
            d.first = (i == 0);
            d.last = (i + 1 == npasses);
            d.seg_rows = plan->sched.segment_rows
                             ? plan->sched.segment_rows
                             : default_seg_rows(plan, d.steps, d.last, ppl, lds);
            hipError_t e = tsq::launch_pass(plan->p.dtype, d, s);
            if (e != hipSuccess)
                return fail(TSQ_ERR_DEVICE, "step pass launch: %s", hipGetErrorString(e));
        }
    }
    if (copy_back) {
        hipError_t e = hipMemcpyAsync(psi, buf[1], plan->sites * plan->elem, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "copy back: %s", hipGetErrorString(e));
    }
    return ok();
}

int tsq_observables(const tsq_plan* plan, const void* psi, const double* V, double* norm_out,
                    double* energy_out, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !psi || !V || !norm_out || !energy_out) return fail(TSQ_ERR_ARG, "null argument");
    int rc = check_ws(plan, ws, ws_bytes);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* scratch = reinterpret_cast<double*>(static_cast<char*>(ws) + plan->off_scratch);
    double* result = scratch + 2 * tsq::kReduceBlocks;
    const int nblocks = plan->p.ny < tsq::kReduceBlocks ? plan->p.ny : tsq::kReduceBlocks;
    hipError_t e = tsq::launch_observables(plan->p.dtype, psi, V, plan->p.nx, plan->p.ny, plan->Jx,
                                           plan->Jy, plan->eps0, scratch, nblocks, result, s);
    if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "observables launch: %s", hipGetErrorString(e));
    double host[2];
    e = hipMemcpyAsync(host, result, sizeof host, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "observables: %s", hipGetErrorString(e));
    *norm_out = host[0];
    *energy_out = host[1];
    return ok();
}

}  // extern "C"
