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
#include <algorithm>
#include <map>
#include <utility>
#include <vector>

#include "../../include/tsq.h"
#include "tsq_internal.h"
#include "tsq_internal3.h"

// One kind of second-order sub-step: its duration, rotation coefficients and
// phase table.  Order 2 has one kind (dt); order 4 has two (p dt, (1-4p) dt).
struct SubStep {
    double dt;
    tsq::Coef64 oxh, oyh, ox2, oy2;  // tau = dt/2 and tau = dt along x, y
    size_t off_ptab;
};

struct tsq_plan {
    tsq_problem p;
    double Jx, Jy, Jz, eps0;
    bool three_d;                    // nz >= 2
    tsq::Coef64 ozh, oz2;            // z factors of a 3D mesh, tau = dt/2 and dt
    tsq::Coef64 oxh, oyh, ox2, oy2;   // of kind 0
    int nkinds;
    SubStep kind[2];
    tsq_schedule sched;   // resolved (segment_rows may stay 0 = per launch)
    size_t sites, elem, pelem;
    size_t off_psi2, off_ptab, off_scratch, off_turns, ws_bytes;
    const void* ws_bound;
    bool td;  // the bound workspace holds a time-dependent table (tsq_set_potential_td)
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
    return tsq::Coef64{std::sin(al), 2.0 * h * h, al};
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Largest rotation angle of a whole time step (|dt| J / hbar) a periodic 2D
// plan accepts: tan of it stays below 1.6.
constexpr double kMaxAngle = 1.0;

constexpr size_t kScratchBytes = (2 * tsq::kReduceBlocks + 2) * sizeof(double);

// Default schedule.  Steps per pass: 5 with the register phase ring (within a
// few percent of the fastest schedule for both dtypes at 4096^2).  Segment
// height: as many wavefront tiles as the device holds resident at once (one
// round, no tail of a partly filled second round), each segment at least 2K
// row pairs long so the discarded warm-up pairs stay below half the work.
constexpr int kDefaultSteps = 5;

// Fill the zero fields of a requested schedule with defaults; false if the
// combination has no kernel instance.
bool resolve_schedule(const tsq_schedule& in, tsq_schedule& out) {
    out = in;
    if (out.steps_per_pass == 0) out.steps_per_pass = kDefaultSteps;
    if (out.phase_store == 0) out.phase_store = out.steps_per_pass <= tsq::kMaxRegSteps ? 1 : 2;
    if (out.pairs_per_lane == 0) out.pairs_per_lane = 1;
    if (out.phase_store == 1 && out.steps_per_pass > tsq::kMaxRegSteps) return false;
    if (out.phase_store == 1 && out.pairs_per_lane == 2 && out.steps_per_pass > tsq::kMaxRegSteps2)
        return false;
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

int occupancy_cached(int dtype, int steps, bool last, int ppl, bool lds, bool closed, bool td,
                     bool u4 = false) {
    // [dtype][steps][last][ppl][lds][closed][td][u4]; 0 = not yet queried
    static std::atomic<int> table[2][tsq::kMaxSteps + 1][2][3][2][2][2][2];
    std::atomic<int>& slot = table[dtype & 1][steps][last ? 1 : 0][ppl][lds ? 1 : 0][closed ? 1 : 0]
                                  [td ? 1 : 0][u4 ? 1 : 0];
    int v = slot.load(std::memory_order_relaxed);
    if (v == 0) {
        v = tsq::march_blocks_per_cu(dtype, steps, last, ppl, lds, false, closed, td, u4);
        if (v <= 0) v = 1;
        slot.store(v, std::memory_order_relaxed);
    }
    return v;
}

int default_seg_rows(const tsq_plan* p, int steps, bool last, int ppl, bool lds, bool closed,
                     bool td, bool u4 = false) {
    const tsq::MarchGeometry g = tsq::march_geometry(p->p.nx, p->p.ny, steps, last, ppl, 2);
    int cus = device_cus();
    if (cus <= 0) cus = 256;
    const long long slots =
        (long long)cus * occupancy_cached(p->p.dtype, steps, last, ppl, lds, closed, td, u4) *
        tsq::kWavesPerBlock;
    const long long pairs = (p->p.ny + 1) / 2;
    // a launch has one block per segment of kWavesPerBlock strips
    const long long strip_slots =
        (g.nstrips + tsq::kWavesPerBlock - 1) / tsq::kWavesPerBlock * tsq::kWavesPerBlock;
    long long segs = slots / strip_slots;
    if (segs < 1) segs = 1;
    if (segs > pairs) segs = pairs;
    long long pairs_per_seg = (pairs + segs - 1) / segs;
    const long long min_pairs = 2LL * (steps + (last ? 1 : 0));
    if (pairs_per_seg < min_pairs) pairs_per_seg = min_pairs;
    return (int)(2 * pairs_per_seg);
}

// Fourth order on a periodic 2D mesh runs one pass per fourth-order step (its
// five sub-steps fused, both phase tables read in the pass).
bool fused_order4(const tsq_plan* p) {
    return p->p.order == 4 && !p->three_d && p->p.bc == TSQ_BC_PERIODIC;
}

// -2 log of the scale the phase table of sub-step kind k carries: on periodic
// 2D meshes the cosines of a steady step of that kind (the tangent-form factors
// leave them out), from the tangents rounded in the plan's dtype; else 0.
double table_log(const tsq_plan* p, int k) {
    if (p->three_d || p->p.bc != TSQ_BC_PERIODIC) return 0.0;
    const SubStep& u = p->kind[k];
    return p->p.dtype == TSQ_C128 ? tsq::step_log_sec2<double>(u.oxh, u.oyh, u.ox2, u.oy2)
                                  : tsq::step_log_sec2<float>(u.oxh, u.oyh, u.ox2, u.oy2);
}

// Closed 2D meshes: log(1 + t^2) of the even x and y tangents of sub-step
// kind k as the march rounds them (the squared secant each even factor
// multiplies a paired site by).
void closed_even_logs(const tsq_plan* p, int k, double& Lx, double& Ly) {
    const SubStep& u = p->kind[k];
    const bool c128 = p->p.dtype == TSQ_C128;
    Lx = c128 ? tsq::log_sec2(tsq::tangent<double>(u.oxh)) : tsq::log_sec2(tsq::tangent<float>(u.oxh));
    Ly = c128 ? tsq::log_sec2(tsq::tangent<double>(u.oyh)) : tsq::log_sec2(tsq::tangent<float>(u.oyh));
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

// Passes of one evolution as groups of equal passes.  A group's passes all
// apply `size` sub-steps of one kind; `opens` marks that its first pass starts
// a run of that kind (opening odd factor of half length), `closes` that its
// last pass ends the run (closing odd factor).  Order 2 is one run of `steps`
// sub-steps; order 4 is U2(p)^2 U2(m) U2(p)^2 per step, so runs alternate
// between 2 or 4 p sub-steps (neighbouring steps share theirs) and 1 m sub-step.
struct PassGroup {
    int kind;
    int size;
    int64_t count;
    bool opens, closes;
};

bool pass_groups(const tsq_plan* p, int64_t steps, int S, std::vector<PassGroup>& g) {
    g.clear();
    auto add_run = [&](int kind, int64_t count) {
        const int64_t full = count / S;
        const int rem = (int)(count % S);
        if (full > 0) g.push_back(PassGroup{kind, S, full, true, rem == 0});
        if (rem > 0) g.push_back(PassGroup{kind, rem, 1, full == 0, true});
    };
    if (steps <= 0) return false;
    if (p->p.order == 4) {
        add_run(0, 2);
        for (int64_t i = 0; i < steps; ++i) {
            add_run(1, 1);
            add_run(0, i + 1 < steps ? 4 : 2);
        }
    } else {
        add_run(0, steps);
    }
    int64_t total = 0;
    for (const PassGroup& x : g) total += x.count;
    if (!(total & 1)) return false;
    for (size_t i = g.size(); i-- > 0;) {
        if (g[i].size < 2) continue;
        const PassGroup o = g[i];
        const int a = o.size / 2, b = o.size - a;
        std::vector<PassGroup> tail(g.begin() + i + 1, g.end());
        g.resize(i);
        if (o.count > 1) g.push_back(PassGroup{o.kind, o.size, o.count - 1, o.opens, false});
        g.push_back(PassGroup{o.kind, a, 1, o.count > 1 ? false : o.opens, false});
        g.push_back(PassGroup{o.kind, b, 1, false, o.closes});
        g.insert(g.end(), tail.begin(), tail.end());
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

}  // extern "C"

// ---------------------------------------------------------------- batched form (host side)

struct BatchLaunch {
    int steps;
    bool last;
    size_t jobs_off;
    int njobs;
    size_t tiles_off;
    int ntiles;
    int nwaves;
};

struct BatchCopy {
    void* dst;
    const void* src;
    size_t bytes;
};

struct tsq_batch {
    int dtype = 0;
    tsq_schedule sched{};
    std::vector<BatchLaunch> launches;
    std::vector<BatchCopy> copies;
    std::vector<unsigned char> blob;  // host image of the device work lists
    char* bws = nullptr;              // device copy (after upload)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t total_tiles = 0;
};

namespace {

size_t blob_reserve(std::vector<unsigned char>& blob, size_t bytes) {
    const size_t off = align_up(blob.size(), 256);
    blob.resize(off + bytes);
    return off;
}

template <class R>
void append_launch(tsq_batch* b, int steps, bool last, const std::vector<tsq::PassDesc>& descs,
                   int slots) {
    const int ppl = b->sched.pairs_per_lane;
    const int K = steps + (last ? 1 : 0);
    // Tile height: the schedule's segment_rows if set; else the strips of all
    // problems stacked, cut into about one tile per resident wavefront, never
    // shorter than 2K row pairs.
    long long h = b->sched.segment_rows;
    if (h <= 0) {
        long long strip_rows = 0;
        for (const tsq::PassDesc& d : descs)
            strip_rows +=
                (long long)tsq::march_geometry(d.nx, d.ny, steps, last, ppl, 2).nstrips * d.ny;
        h = (strip_rows + slots - 1) / slots;
        if (h < 4LL * K) h = 4LL * K;
        h = (h + 1) & ~1LL;
    }

    std::vector<tsq::MarchArgs<R>> jobs;
    std::vector<tsq::BatchTile> tiles;
    for (size_t j = 0; j < descs.size(); ++j) {
        tsq::PassDesc d = descs[j];
        d.seg_rows = (int)std::min<long long>(h, d.ny);
        const tsq::MarchGeometry g = tsq::march_geometry(d.nx, d.ny, steps, last, ppl, d.seg_rows);
        jobs.push_back(tsq::make_march_args<R>(d, g));
        for (int st = 0; st < g.nstrips; ++st)
            for (int sg = 0; sg < g.nsegs; ++sg) {
                const int rows = std::min(d.seg_rows, d.ny - sg * d.seg_rows);
                tiles.push_back(tsq::BatchTile{(int)j, st, sg, rows});
            }
    }
    std::stable_sort(tiles.begin(), tiles.end(),
                     [](const tsq::BatchTile& x, const tsq::BatchTile& y) { return x.rows > y.rows; });
    BatchLaunch L;
    L.steps = steps;
    L.last = last;
    L.njobs = (int)jobs.size();
    L.ntiles = (int)tiles.size();
    L.nwaves = std::min(L.ntiles, slots);
    L.jobs_off = blob_reserve(b->blob, jobs.size() * sizeof(tsq::MarchArgs<R>));
    std::memcpy(b->blob.data() + L.jobs_off, jobs.data(), jobs.size() * sizeof(tsq::MarchArgs<R>));
    L.tiles_off = blob_reserve(b->blob, tiles.size() * sizeof(tsq::BatchTile));
    std::memcpy(b->blob.data() + L.tiles_off, tiles.data(), tiles.size() * sizeof(tsq::BatchTile));
    b->launches.push_back(L);
    b->total_tiles += L.ntiles;
}

int enqueue_batch(tsq_batch* b, hipStream_t s) {
    const bool lds = b->sched.phase_store == 2;
    for (const BatchLaunch& L : b->launches) {
        hipError_t e = tsq::launch_batch(b->dtype, L.steps, L.last, b->sched.pairs_per_lane, lds,
                                         b->bws + L.jobs_off,
                                         reinterpret_cast<const tsq::BatchTile*>(b->bws + L.tiles_off),
                                         L.ntiles, L.nwaves, s);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "batched pass launch: %s", hipGetErrorString(e));
    }
    for (const BatchCopy& c : b->copies) {
        hipError_t e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "batch copy back: %s", hipGetErrorString(e));
    }
    return TSQ_OK;
}

void drop_graph(tsq_batch* b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

extern "C" {

int tsq_batch_create(tsq_plan* const* plans, void* const* psi, void* const* ws, const int64_t* steps,
                     int32_t n, const tsq_schedule* schedule, tsq_batch** out) {
    if (!plans || !psi || !ws || !steps || !out || n < 1)
        return fail(TSQ_ERR_ARG, "null argument or empty batch");
    const int dtype = plans[0] ? plans[0]->p.dtype : -1;
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !psi[i] || !ws[i]) return fail(TSQ_ERR_ARG, "null entry %d", i);
        if (steps[i] < 0) return fail(TSQ_ERR_ARG, "steps[%d] = %lld < 0", i, (long long)steps[i]);
        if (plans[i]->p.dtype != dtype) return fail(TSQ_ERR_DTYPE, "batch mixes dtypes (entry %d)", i);
        if (plans[i]->p.order != 2 || plans[i]->p.bc != TSQ_BC_PERIODIC || plans[i]->three_d)
            return fail(TSQ_ERR_UNSUPPORTED,
                        "entry %d: the batched form runs periodic order-2 2D plans only", i);
        if (plans[i]->ws_bound != ws[i])
            return fail(TSQ_ERR_STATE, "entry %d: workspace is not the one given to tsq_set_potential", i);
        if (plans[i]->td)
            return fail(TSQ_ERR_UNSUPPORTED,
                        "entry %d: the batched form runs time-independent potentials only", i);
        if (reinterpret_cast<uintptr_t>(psi[i]) % 16 != 0)
            return fail(TSQ_ERR_ARG, "entry %d: psi must be 16-byte aligned", i);
    }
    const tsq_schedule want = schedule ? *schedule : tsq_schedule{0, 0, 0, 0};
    tsq_schedule sc;
    if (want.steps_per_pass < 0 || want.steps_per_pass > tsq::kMaxSteps || want.pairs_per_lane < 0 ||
        want.pairs_per_lane > 2 || want.phase_store < 0 || want.phase_store > 2 ||
        want.segment_rows < 0 || (want.segment_rows & 1) || !resolve_schedule(want, sc))
        return fail(TSQ_ERR_ARG, "invalid batch schedule");
    int cus = device_cus();
    if (cus <= 0) return fail(TSQ_ERR_DEVICE, "no device to size the batch for");

    // passes of every problem
    std::vector<std::vector<int>> sizes(n);
    int64_t maxp = 0, total = 0;
    tsq_batch* b = new (std::nothrow) tsq_batch();
    if (!b) return fail(TSQ_ERR_ARG, "out of host memory");
    b->dtype = dtype;
    b->sched = sc;
    for (int i = 0; i < n; ++i) {
        std::vector<Run> runs;
        const bool cb = steps[i] > 0 && pass_runs(steps[i], sc.steps_per_pass, runs);
        total += run_passes(runs);
        if (total > 50000000LL) {
            delete b;
            return fail(TSQ_ERR_ARG, "batch of %lld passes is too large", (long long)total);
        }
        for (const Run& r : runs)
            for (int64_t k = 0; k < r.count; ++k) sizes[i].push_back(r.size);
        maxp = std::max<int64_t>(maxp, (int64_t)sizes[i].size());
        if (cb) {
            char* w = static_cast<char*>(ws[i]);
            b->copies.push_back(BatchCopy{psi[i], w + plans[i]->off_psi2, plans[i]->sites * plans[i]->elem});
        }
    }
    const bool lds = sc.phase_store == 2;
    for (int64_t l = 0; l < maxp; ++l) {
        std::map<std::pair<int, bool>, std::vector<tsq::PassDesc>> groups;
        for (int i = 0; i < n; ++i) {
            if ((int64_t)sizes[i].size() <= l) continue;
            const tsq_plan* pl = plans[i];
            char* w = static_cast<char*>(ws[i]);
            void* buf[2] = {psi[i], w + pl->off_psi2};
            tsq::PassDesc d;
            d.src = buf[l & 1];
            d.dst = buf[(l + 1) & 1];
            d.ptab = w + pl->off_ptab;
            d.nx = pl->p.nx;
            d.ny = pl->p.ny;
            d.steps = sizes[i][l];
            d.first = (l == 0);
            d.last = (l + 1 == (int64_t)sizes[i].size());
            d.seg_rows = 2;
            d.pairs_per_lane = sc.pairs_per_lane;
            d.phase_lds = lds;
            d.oxh = pl->oxh;
            d.oyh = pl->oyh;
            d.ox2 = pl->ox2;
            d.oy2 = pl->oy2;
            groups[{d.steps, d.last}].push_back(d);
        }
        for (auto& kv : groups) {
            const int st = kv.first.first;
            const bool last = kv.first.second;
            int bpc = tsq::march_blocks_per_cu(dtype, st, last, sc.pairs_per_lane, lds, true);
            if (bpc <= 0) bpc = 1;
            const int slots = cus * bpc * tsq::kWavesPerBlock;
            if (dtype == TSQ_C128)
                append_launch<double>(b, st, last, kv.second, slots);
            else
                append_launch<float>(b, st, last, kv.second, slots);
        }
    }
    *out = b;
    return ok();
}

int tsq_batch_destroy(tsq_batch* b) {
    if (b) drop_graph(b);
    delete b;
    return ok();
}

int tsq_batch_workspace_size(const tsq_batch* b, size_t* bytes) {
    if (!b || !bytes) return fail(TSQ_ERR_ARG, "null argument");
    *bytes = align_up(b->blob.size(), 256) + 256;
    return ok();
}

int tsq_batch_info(const tsq_batch* b, int64_t* launches, int64_t* tiles) {
    if (!b || !launches || !tiles) return fail(TSQ_ERR_ARG, "null argument");
    *launches = (int64_t)b->launches.size();
    *tiles = b->total_tiles;
    return ok();
}

int tsq_batch_upload(tsq_batch* b, void* bws, size_t bytes, void* stream) {
    if (!b || !bws) return fail(TSQ_ERR_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(bws) % 256 != 0)
        return fail(TSQ_ERR_WORKSPACE, "batch workspace must be 256-byte aligned");
    size_t need = 0;
    tsq_batch_workspace_size(b, &need);
    if (bytes < need)
        return fail(TSQ_ERR_WORKSPACE, "batch workspace of %zu bytes is smaller than %zu", bytes, need);
    if (b->bws != bws) drop_graph(b);
    hipError_t e = hipMemcpyAsync(bws, b->blob.data(), b->blob.size(), hipMemcpyHostToDevice,
                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "batch upload: %s", hipGetErrorString(e));
    b->bws = static_cast<char*>(bws);
    return ok();
}

int tsq_batch_launch(tsq_batch* b, int32_t use_graph, void* stream) {
    if (!b) return fail(TSQ_ERR_ARG, "null batch");
    if (!b->bws) return fail(TSQ_ERR_STATE, "tsq_batch_upload has not been called");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!use_graph) {
        int rc = enqueue_batch(b, s);
        return rc ? rc : ok();
    }
    if (!b->exec) {
        if (s == nullptr) return fail(TSQ_ERR_ARG, "graph capture needs a non-null stream");
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "begin capture: %s", hipGetErrorString(e));
        int rc = enqueue_batch(b, s);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e2 != hipSuccess) return fail(TSQ_ERR_DEVICE, "end capture: %s", hipGetErrorString(e2));
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return fail(TSQ_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
        }
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "graph launch: %s", hipGetErrorString(e));
    return ok();
}

int tsq_batch_evolve_workspace_size(tsq_plan* const* plans, void* const* psi, void* const* ws,
                                    const int64_t* steps, int32_t n, const tsq_schedule* schedule,
                                    size_t* bytes) {
    if (!bytes) return fail(TSQ_ERR_ARG, "null output pointer");
    tsq_batch* b = nullptr;
    int rc = tsq_batch_create(plans, psi, ws, steps, n, schedule, &b);
    if (rc) return rc;
    tsq_batch_workspace_size(b, bytes);
    delete b;
    return ok();
}

int tsq_batch_evolve(tsq_plan* const* plans, void* const* psi, void* const* ws, const int64_t* steps,
                     int32_t n, const tsq_schedule* schedule, void* bws, size_t bws_bytes,
                     void* stream) {
    return tsq::batch_evolve_into(plans, psi, ws, steps, n, schedule, bws, bws_bytes, stream,
                                  nullptr);
}

const char* tsq_last_error(void) { return g_err.c_str(); }

}  // extern "C"

int tsq::set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int tsq::batch_evolve_into(tsq_plan* const* plans, void* const* psi, void* const* ws,
                           const int64_t* steps, int32_t n, const tsq_schedule* schedule,
                           void* bws, size_t bws_bytes, void* stream, size_t* need) {
    tsq_batch* b = nullptr;
    int rc = tsq_batch_create(plans, psi, ws, steps, n, schedule, &b);
    if (rc) return rc;
    if (need) tsq_batch_workspace_size(b, need);
    rc = tsq_batch_upload(b, bws, bws_bytes, stream);
    if (!rc) rc = tsq_batch_launch(b, 0, stream);
    // the upload reads pageable host memory, which the copy has staged by the
    // time it returns; the host image is kept until the thread's next call anyway
    thread_local std::vector<unsigned char> keep;
    keep.swap(b->blob);
    delete b;
    return rc ? rc : ok();
}

extern "C" {

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
    if (pr->order != 0 && pr->order != 2 && pr->order != 4)
        return fail(TSQ_ERR_ARG, "order must be 2 or 4 (got %d)", pr->order);
    const bool three_d = pr->nz >= 2;
    if (pr->nz < 0) return fail(TSQ_ERR_SHAPE, "nz must be >= 0 (got %d)", pr->nz);
    if (three_d) {
        if (!finite_pos(pr->dz)) return fail(TSQ_ERR_ARG, "dz must be finite and > 0 (%g)", pr->dz);
        if (pr->bc != TSQ_BC_PERIODIC)
            return fail(TSQ_ERR_UNSUPPORTED, "3D meshes run with periodic boundaries only");
        if (pr->order == 4) return fail(TSQ_ERR_UNSUPPORTED, "3D meshes run the order-2 step only");
        if (pr->nz & 1)
            return fail(TSQ_ERR_SHAPE, "nz = %d: periodic boundaries need even sides", pr->nz);
        if ((long long)pr->nx * (long long)pr->ny * (long long)pr->nz > 0x7fffffffLL)
            return fail(TSQ_ERR_SHAPE, "mesh %d x %d x %d exceeds 2^31-1 sites", pr->nx, pr->ny,
                        pr->nz);
    }

    tsq_plan* p = new (std::nothrow) tsq_plan();
    if (!p) return fail(TSQ_ERR_ARG, "out of host memory");
    p->p = *pr;
    const double hb = pr->hbar, m = pr->mass;
    p->Jx = hb * hb / (2.0 * m * pr->dx * pr->dx);
    p->Jy = hb * hb / (2.0 * m * pr->dy * pr->dy);
    p->eps0 = hb * hb / (m * pr->dx * pr->dx) + hb * hb / (m * pr->dy * pr->dy);
    p->three_d = three_d;
    p->Jz = 0.0;
    if (three_d) {
        p->Jz = hb * hb / (2.0 * m * pr->dz * pr->dz);
        p->eps0 += hb * hb / (m * pr->dz * pr->dz);
        p->ozh = block_coef(0.5 * pr->dt, p->Jz, hb);
        p->oz2 = block_coef(pr->dt, p->Jz, hb);
    } else {
        p->p.nz = 1;
    }
    if (p->p.order == 0) p->p.order = 2;
    double dts[2] = {pr->dt, 0.0};
    p->nkinds = 1;
    if (p->p.order == 4) {
        const double q = 1.0 / (4.0 - std::cbrt(4.0));
        dts[0] = q * pr->dt;
        dts[1] = (1.0 - 4.0 * q) * pr->dt;
        p->nkinds = 2;
    }
    for (int k = 0; k < p->nkinds; ++k) {
        SubStep& u = p->kind[k];
        u.dt = dts[k];
        u.oxh = block_coef(0.5 * dts[k], p->Jx, hb);
        u.oyh = block_coef(0.5 * dts[k], p->Jy, hb);
        u.ox2 = block_coef(dts[k], p->Jx, hb);
        u.oy2 = block_coef(dts[k], p->Jy, hb);
    }
    // Periodic 2D meshes rotate in the tangent form (tan al of the half and
    // whole time step), closed ones their even factors (half step), which
    // needs every such angle well inside (-pi/2, pi/2).
    if (!three_d) {
        const bool closed = pr->bc == TSQ_BC_CLOSED;
        const double limit = closed ? 2.0 * kMaxAngle : kMaxAngle;  // on the whole-step angle
        for (int k = 0; k < p->nkinds; ++k) {
            const SubStep& u = p->kind[k];
            if (std::fabs(u.ox2.al) >= limit || std::fabs(u.oy2.al) >= limit) {
                delete p;
                return fail(TSQ_ERR_UNSUPPORTED,
                            "|dt| hbar / (2 m da^2) = %g rad per step along %s is too large for the "
                            "tangent-form rotation of %s meshes (limit %g)",
                            std::max(std::fabs(u.ox2.al), std::fabs(u.oy2.al)),
                            std::fabs(u.ox2.al) >= std::fabs(u.oy2.al) ? "x" : "y",
                            closed ? "closed" : "periodic", limit);
            }
        }
    }
    p->oxh = p->kind[0].oxh;
    p->oyh = p->kind[0].oyh;
    p->ox2 = p->kind[0].ox2;
    p->oy2 = p->kind[0].oy2;
    resolve_schedule(tsq_schedule{0, 0, 0, 0}, p->sched);
    p->sites = (size_t)pr->nx * (size_t)pr->ny * (size_t)p->p.nz;
    p->elem = pr->dtype == TSQ_C128 ? 16 : 8;
    // bytes per site of a phase-table area: complex128 exp(-i phi) (16);
    // complex64 uses 8 (two 32-bit fixed-point parts) and the time-dependent
    // table of either dtype 16, so the area keeps 16
    p->pelem = 16;
    p->off_psi2 = 0;
    p->off_ptab = align_up(p->sites * p->elem, 256);
    size_t end = p->off_ptab;
    for (int k = 0; k < p->nkinds; ++k) {
        p->kind[k].off_ptab = end;
        end = align_up(end + p->sites * p->pelem, 256);
    }
    p->off_scratch = end;
    // the time-dependent phase's kTurns factors (double2)
    p->off_turns = align_up(p->off_scratch + kScratchBytes, 256);
    p->ws_bytes = p->off_turns + tsq::kTurns * 16;
    p->ws_bound = nullptr;
    p->td = false;
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
                    "(registers hold at most %d steps, %d with 2 pairs per lane; LDS needs 1 "
                    "pair per lane)",
                    r.steps_per_pass, r.pairs_per_lane, r.phase_store, tsq::kMaxRegSteps,
                    tsq::kMaxRegSteps2);
    if (plan->p.bc == TSQ_BC_CLOSED && r.pairs_per_lane != 1)
        return fail(TSQ_ERR_ARG, "closed meshes run with 1 pair per lane");
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
    if (plan->p.order == 4 && steps > 10000000LL)
        return fail(TSQ_ERR_ARG, "order-4 evolution of %lld steps is too long for one call",
                    (long long)steps);
    if (plan->three_d) {  // one step per pass, then a closing pass
        *passes = steps > 0 ? steps + 1 : 0;
        *copy_back = (steps > 0 && !(steps & 1)) ? 1 : 0;
        return ok();
    }
    if (fused_order4(plan)) {  // one pass per fourth-order step
        *passes = steps;
        *copy_back = (steps & 1) ? 1 : 0;
        return ok();
    }
    std::vector<PassGroup> groups;
    const int S = plan->td ? std::min(plan->sched.steps_per_pass, tsq::kMaxTdSteps)
                           : plan->sched.steps_per_pass;
    const bool cb = pass_groups(plan, steps, S, groups);
    int64_t n = 0;
    for (const PassGroup& x : groups) n += x.count;
    *passes = n;
    *copy_back = cb ? 1 : 0;
    return ok();
}

int tsq_set_potential(tsq_plan* plan, const double* V, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !V) return fail(TSQ_ERR_ARG, "null plan or potential");
    int rc = check_ws(plan, ws, ws_bytes);
    if (rc) return rc;
    char* w = static_cast<char*>(ws);
    for (int k = 0; k < plan->nkinds; ++k) {
        const SubStep& u = plan->kind[k];
        // 2D meshes: the table carries the cosines the march's tangent-form
        // factors leave out, a step's on periodic meshes, the even factors'
        // that pair the site on closed ones
        tsq::TableScale scale;
        if (!plan->three_d && plan->p.bc == TSQ_BC_CLOSED) {
            double Lx, Ly;
            closed_even_logs(plan, k, Lx, Ly);
            // two even x and two even y factors per step: cos^2 = exp(-log_sec2)
            scale.g = std::exp(-(Lx + Ly));
            scale.gx = std::exp(-Ly);
            scale.gy = std::exp(-Lx);
            scale.gxy = 1.0;
            scale.nx = plan->p.nx;
            scale.wx = (plan->p.nx & 1) ? plan->p.nx - 1 : -1;
            scale.wy0 = (plan->p.ny & 1) ? (long long)(plan->p.ny - 1) * plan->p.nx : -1;
        } else {
            scale.g = std::exp(-0.5 * table_log(plan, k));
        }
        hipError_t e = tsq::launch_phase_table(plan->p.dtype, V, w + u.off_ptab,
                                               (long long)plan->sites, u.dt, plan->eps0,
                                               plan->p.hbar, scale,
                                               static_cast<hipStream_t>(stream));
        if (e != hipSuccess)
            return fail(TSQ_ERR_DEVICE, "phase table launch: %s", hipGetErrorString(e));
    }
    plan->ws_bound = ws;
    plan->td = false;
    return ok();
}

int tsq_set_potential_td(tsq_plan* plan, const double* V0, const double* W, void* ws,
                         size_t ws_bytes, void* stream) {
    if (!plan || !V0 || !W) return fail(TSQ_ERR_ARG, "null plan or potential");
    if (plan->p.order != 2)
        return fail(TSQ_ERR_UNSUPPORTED, "time-dependent potentials run with order-2 plans only");
    if (plan->three_d)
        return fail(TSQ_ERR_UNSUPPORTED, "time-dependent potentials run on 2D meshes only");
    int rc = check_ws(plan, ws, ws_bytes);
    if (rc) return rc;
    char* w = static_cast<char*>(ws);
    // the factors carry the cosines the tangent-form rotations leave out, as the
    // static table does: a step's on periodic meshes, the four even factors' on
    // closed ones (the march rescales the last odd column and row)
    double scale = std::exp(-0.5 * table_log(plan, 0));
    if (plan->p.bc == TSQ_BC_CLOSED) {
        double Lx, Ly;
        closed_even_logs(plan, 0, Lx, Ly);
        scale = std::exp(-(Lx + Ly));
    }
    hipError_t e = tsq::launch_td_table(V0, W, w + plan->kind[0].off_ptab, w + plan->off_turns,
                                        (long long)plan->sites, plan->kind[0].dt, plan->eps0,
                                        plan->p.hbar, scale, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "table launch: %s", hipGetErrorString(e));
    plan->ws_bound = ws;
    plan->td = true;
    return ok();
}

}  // extern "C"

namespace {

// Checks shared by tsq_evolve and tsq_evolve_td.
int check_evolve(const tsq_plan* plan, const void* psi, int64_t steps, const void* ws,
                 size_t ws_bytes) {
    if (!plan || !psi) return fail(TSQ_ERR_ARG, "null plan or psi");
    if (steps < 0) return fail(TSQ_ERR_ARG, "steps must be >= 0 (%lld)", (long long)steps);
    if (reinterpret_cast<uintptr_t>(psi) % 16 != 0) return fail(TSQ_ERR_ARG, "psi must be 16-byte aligned");
    int rc = check_ws(plan, ws, ws_bytes);
    if (rc) return rc;
    if (plan->ws_bound == nullptr) return fail(TSQ_ERR_STATE, "tsq_set_potential has not been called");
    if (plan->ws_bound != ws)
        return fail(TSQ_ERR_STATE, "workspace differs from the one given to tsq_set_potential");
    if (plan->p.order == 4 && steps > 10000000LL)
        return fail(TSQ_ERR_ARG, "order-4 evolution of %lld steps is too long for one call",
                    (long long)steps);
    return TSQ_OK;
}

// Fourth order on a periodic 2D mesh: one pass per step, sub-steps p, p, m,
// p, p with both phase tables; an odd pass count ends with a copy back.
int run_evolution_order4(tsq_plan* plan, void* psi, int64_t steps, void* ws, hipStream_t s) {
    char* w = static_cast<char*>(ws);
    void* buf[2] = {psi, w + plan->off_psi2};
    tsq::PassDesc d;
    d.nx = plan->p.nx;
    d.ny = plan->p.ny;
    d.pairs_per_lane = 1;
    d.phase_lds = true;
    d.u4 = true;
    d.steps = 5;
    const SubStep& p = plan->kind[0];
    const SubStep& m = plan->kind[1];
    d.ptab = w + p.off_ptab;
    d.ptab2 = w + m.off_ptab;
    d.oxh = p.oxh;
    d.oyh = p.oyh;
    d.ox2 = p.ox2;
    d.oy2 = p.oy2;
    d.mxh = m.oxh;
    d.myh = m.oyh;
    d.log_table_p = table_log(plan, 0);
    d.log_table_m = table_log(plan, 1);
    for (int64_t i = 0; i < steps; ++i) {
        d.src = buf[i & 1];
        d.dst = buf[(i + 1) & 1];
        d.first = i == 0;
        d.last = i + 1 == steps;
        d.seg_rows = plan->sched.segment_rows
                         ? plan->sched.segment_rows
                         : default_seg_rows(plan, 5, d.last, 1, true, false, false, true);
        hipError_t e = tsq::launch_pass(plan->p.dtype, d, s);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "order-4 pass launch: %s", hipGetErrorString(e));
    }
    if (steps & 1) {
        hipError_t e = hipMemcpyAsync(psi, buf[1], plan->sites * plan->elem, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "copy back: %s", hipGetErrorString(e));
    }
    return ok();
}

// Launch the passes of `steps` steps (f: per-step modulation of a
// time-dependent potential, else null) and the copy back if any.
int run_evolution(tsq_plan* plan, void* psi, int64_t steps, void* ws, hipStream_t s,
                  const double* f) {
    if (!f && fused_order4(plan)) return run_evolution_order4(plan, psi, steps, ws, s);
    char* w = static_cast<char*>(ws);
    void* buf[2] = {psi, w + plan->off_psi2};
    const bool td = f != nullptr;
    const int S = td ? std::min(plan->sched.steps_per_pass, tsq::kMaxTdSteps)
                     : plan->sched.steps_per_pass;
    const int ppl = plan->sched.pairs_per_lane;
    const bool lds = plan->sched.phase_store == 2;
    std::vector<PassGroup> groups;
    const bool copy_back = pass_groups(plan, steps, S, groups);

    tsq::PassDesc d;
    d.nx = plan->p.nx;
    d.ny = plan->p.ny;
    d.pairs_per_lane = ppl;
    d.phase_lds = lds;
    d.closed = plan->p.bc == TSQ_BC_CLOSED;
    d.td = td;
    d.ptab2 = td ? w + plan->off_turns : nullptr;
    int64_t i = 0, n0 = 0;  // pass index, first step of the pass
    for (const PassGroup& g : groups) {
        const SubStep& u = plan->kind[g.kind];
        d.ptab = w + u.off_ptab;
        d.oxh = u.oxh;
        d.oyh = u.oyh;
        d.ox2 = u.ox2;
        d.oy2 = u.oy2;
        for (int64_t k = 0; k < g.count; ++k, ++i) {
            d.src = buf[i & 1];
            d.dst = buf[(i + 1) & 1];
            d.steps = g.size;
            d.first = g.opens && k == 0;
            d.last = g.closes && k + 1 == g.count;
            d.f = td ? f + n0 : nullptr;
            d.seg_rows = plan->sched.segment_rows
                             ? plan->sched.segment_rows
                             : default_seg_rows(plan, d.steps, d.last, ppl, lds, d.closed, td);
            hipError_t e = tsq::launch_pass(plan->p.dtype, d, s);
            if (e != hipSuccess)
                return fail(TSQ_ERR_DEVICE, "step pass launch: %s", hipGetErrorString(e));
            n0 += g.size;
        }
    }
    if (copy_back) {
        hipError_t e = hipMemcpyAsync(psi, buf[1], plan->sites * plan->elem, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "copy back: %s", hipGetErrorString(e));
    }
    return ok();
}

// Three-dimensional mesh: one step per pass.
int run_evolution3(tsq_plan* plan, void* psi, int64_t steps, void* ws, hipStream_t s) {
    char* w = static_cast<char*>(ws);
    void* buf[2] = {psi, w + plan->off_psi2};
    int cus = device_cus();
    if (cus <= 0) cus = 256;
    tsq::Pass3Desc d;
    d.ptab = w + plan->kind[0].off_ptab;
    d.nx = plan->p.nx;
    d.ny = plan->p.ny;
    d.nz = plan->p.nz;
    d.oh[0] = plan->oxh;
    d.oh[1] = plan->oyh;
    d.oh[2] = plan->ozh;
    d.o2[0] = plan->ox2;
    d.o2[1] = plan->oy2;
    d.o2[2] = plan->oz2;
    // segment height: at most one tile per CU (tiles = strips x slabs x
    // segments), at least 2 plane pairs; a schedule's segment_rows sets it
    // (segment_rows / 2 plane pairs).  Long segments beat more resident
    // blocks: at 512^3 one segment per column (215 tiles on 256 CUs) runs
    // 1.2x faster than two (430 tiles).
    const long long strips = (d.nx + (tsq::kWaveSize - 2) * 2 - 1) / ((tsq::kWaveSize - 2) * 2);
    const long long slabs = (d.ny / 2 + tsq::kWaves3 - 3) / (tsq::kWaves3 - 2);
    const long long pairs = d.nz / 2;
    long long segs = (long long)cus / (strips * slabs);
    segs = std::max(1LL, std::min(segs, pairs));
    long long per = std::max(2LL, (pairs + segs - 1) / segs);
    if (plan->sched.segment_rows > 0) per = plan->sched.segment_rows / 2;
    d.seg_pairs = (int)std::min(per, pairs);
    // steps passes, then the closing odd factors of the last step
    for (int64_t i = 0; i <= steps; ++i) {
        d.src = buf[i & 1];
        d.dst = buf[(i + 1) & 1];
        d.first = i == 0;
        d.close = i == steps;
        hipError_t e = tsq::launch_pass3(plan->p.dtype, d, s);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "3D pass launch: %s", hipGetErrorString(e));
    }
    if (!(steps & 1)) {  // steps + 1 passes: an odd count ends in the second buffer
        hipError_t e = hipMemcpyAsync(psi, buf[1], plan->sites * plan->elem, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(TSQ_ERR_DEVICE, "copy back: %s", hipGetErrorString(e));
    }
    return ok();
}

}  // namespace

extern "C" {

int tsq_evolve(tsq_plan* plan, void* psi, int64_t steps, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_evolve(plan, psi, steps, ws, ws_bytes);
    if (rc) return rc;
    if (plan->td)
        return fail(TSQ_ERR_STATE, "the workspace holds a time-dependent potential: use tsq_evolve_td");
    if (steps == 0) return ok();
    if (plan->three_d) return run_evolution3(plan, psi, steps, ws, static_cast<hipStream_t>(stream));
    return run_evolution(plan, psi, steps, ws, static_cast<hipStream_t>(stream), nullptr);
}

int tsq_evolve_td(tsq_plan* plan, void* psi, int64_t steps, const double* f, void* ws,
                  size_t ws_bytes, void* stream) {
    int rc = check_evolve(plan, psi, steps, ws, ws_bytes);
    if (rc) return rc;
    if (!plan->td)
        return fail(TSQ_ERR_STATE, "tsq_set_potential_td has not been called on this workspace");
    if (steps > 0 && !f) return fail(TSQ_ERR_ARG, "null modulation array");
    for (int64_t n = 0; n < steps; ++n)
        if (!std::isfinite(f[n])) return fail(TSQ_ERR_ARG, "f[%lld] is not finite", (long long)n);
    if (plan->sched.pairs_per_lane != 1)
        return fail(TSQ_ERR_ARG, "time-dependent potentials run with 1 pair per lane");
    if (steps == 0) return ok();
    return run_evolution(plan, psi, steps, ws, static_cast<hipStream_t>(stream), f);
}

int tsq_observables(const tsq_plan* plan, const void* psi, const double* V, double* norm_out,
                    double* energy_out, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !psi || !V || !norm_out || !energy_out) return fail(TSQ_ERR_ARG, "null argument");
    int rc = check_ws(plan, ws, ws_bytes);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* scratch = reinterpret_cast<double*>(static_cast<char*>(ws) + plan->off_scratch);
    double* result = scratch + 2 * tsq::kReduceBlocks;
    const long long rows = (long long)plan->p.ny * plan->p.nz;
    // 3D: blocks over rows; 2D: the launcher cuts the mesh into at most this many items
    const int nblocks = plan->three_d ? (rows < tsq::kReduceBlocks ? (int)rows : tsq::kReduceBlocks)
                                      : tsq::kReduceBlocks;
    hipError_t e = plan->three_d
                       ? tsq::launch_observables3(plan->p.dtype, psi, V, plan->p.nx, plan->p.ny,
                                                  plan->p.nz, plan->Jx, plan->Jy, plan->Jz,
                                                  plan->eps0, scratch, nblocks, result, s)
                       : tsq::launch_observables(plan->p.dtype, psi, V, plan->p.nx, plan->p.ny,
                                                 plan->Jx, plan->Jy, plan->eps0,
                                                 plan->p.bc == TSQ_BC_CLOSED, scratch, nblocks,
                                                 result, s);
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
