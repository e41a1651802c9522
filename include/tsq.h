/*
 * tsq.h — C ABI of the MI355X (gfx950) second-order Trotter-Suzuki solver.
 *
 * The library evolves one quantum particle on a 2D real-space mesh with the
 * second-order Trotter-Suzuki product of Wittek & Cucchietti, "A Second-Order
 * Distributed Trotter-Suzuki Solver with a Hybrid Kernel" (Sec. 2).  The
 * calls follow the paper's statement of the problem: a mesh of spacing a
 * (Sec. 2, the finite-mesh discretisation), particle mass m and hbar (the
 * Hamiltonian -hbar^2/(2m) d^2/dx^2 + V(x)), the external potential V, the
 * initial state |psi(0)> (Sec. 2, Eq. "evolution"), the time step dt and a
 * number of steps (Sec. 2, the first-order factor U1(dt) and its symmetrised
 * second-order product, Eq. "secondorder").
 *
 * Conventions
 *   - Mesh: nx * ny sites, row-major (y, x), x fastest; a 3D mesh (nz > 1) is
 *     (z, y, x), x fastest, and its step adds the z factors symmetrically:
 *       Ox Oy Oz Ex Ey Ez P Ez Ey Ex Oz Oy Ox, eps0 summing all three axes.  psi is interleaved
 *     complex: complex128 = two doubles (re, im) per site, complex64 = two
 *     floats.  V is one double per site.
 *   - One step is U2(dt) = exp(-i dt H / hbar) + O(dt^3) applied as
 *       Ox(h) Oy(h) Ex(h) Ey(h) P(dt) Ey(h) Ex(h) Oy(h) Ox(h),  h = dt/2,
 *     (first factor applied first) where Ea/Oa rotate the even pairs
 *     (2j, 2j+1) / odd pairs (2j+1, 2j+2) of every line along axis a by the
 *     2x2 block exponential [[cos al, i sin al], [i sin al, cos al]],
 *     al = tau hbar / (2 m da^2), and P multiplies site l by
 *     exp(-i dt (V_l + hbar^2/(m dx^2) + hbar^2/(m dy^2)) / hbar).
 *     Consecutive steps share their odd factors (Ox(h)Ox(h) = Ox(2h)); one
 *     tsq_evolve call therefore applies exactly U2(dt)^steps up to rounding.
 *   - Periodic boundaries: the odd pairs include (L-1, 0); both sides must be
 *     even.  Closed boundaries: hard walls, no pair crosses a wall, sides of
 *     any length >= 2 (the printed H1/H2 of Sec. 2 are of this kind); the
 *     diagonal keeps its full value at the walls.
 *
 * Memory and ownership
 *   - The caller owns all device memory: psi, V, and a workspace of
 *     tsq_workspace_size() bytes (second psi buffer, phase table, reduction
 *     scratch).  The library never allocates or frees device memory and keeps
 *     no device pointer between calls except the workspace address recorded by
 *     tsq_set_potential, which later calls must pass again.
 *   - A plan is host memory owned by the caller (create / destroy).  Plans are
 *     not thread-safe: one thread at a time may use a plan.
 *
 * Streams and errors
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call is asynchronous on that stream except tsq_observables, which
 *     synchronises it to return host values.
 *   - Every function returns a tsq_status; nothing throws or aborts across the
 *     ABI.  Arguments are validated on the host before any launch: a rejected
 *     call launches nothing and leaves every buffer untouched.  A HIP launch
 *     failure is TSQ_ERR_DEVICE with the HIP error string in tsq_last_error().
 *     Asynchronous device faults surface at the next synchronising call.
 */
#ifndef TSQ_H
#define TSQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSQ_ABI_VERSION 5

typedef enum {
    TSQ_OK = 0,
    TSQ_ERR_ARG = -1,         /* null pointer, non-finite or non-positive constant, bad count */
    TSQ_ERR_SHAPE = -2,       /* side < 2, odd side under periodic boundaries, too many sites */
    TSQ_ERR_DTYPE = -3,       /* unknown dtype */
    TSQ_ERR_WORKSPACE = -4,   /* workspace too small or misaligned */
    TSQ_ERR_DEVICE = -5,      /* a HIP call failed; see tsq_last_error() */
    TSQ_ERR_STATE = -6,       /* call out of order (e.g. evolve before set_potential, other ws) */
    TSQ_ERR_UNSUPPORTED = -7  /* valid request the library does not implement */
} tsq_status;

typedef enum { TSQ_C64 = 0, TSQ_C128 = 1 } tsq_dtype;
typedef enum { TSQ_BC_PERIODIC = 0, TSQ_BC_CLOSED = 1 } tsq_bc;

/* The problem statement of Sec. 2: mesh, spacing, mass, hbar, time step. */
typedef struct {
    int32_t nx, ny;   /* sites along x and y; >= 2, even under periodic boundaries */
    double dx, dy;    /* mesh spacing a along each axis; finite, > 0 */
    double mass;      /* particle mass m; finite, > 0 */
    double hbar;      /* reduced Planck constant; finite, > 0 */
    double dt;        /* time step; finite, any sign (negative evolves backwards) */
    int32_t bc;       /* tsq_bc */
    int32_t dtype;    /* tsq_dtype of psi */
    int32_t order;    /* 2: U2(dt) per step (Eq. "secondorder"); 4: U4(dt) per step,
                         U2(p dt)^2 U2((1-4p) dt) U2(p dt)^2, p = 1/(4 - 4^(1/3))
                         (Eq. "fourthorder"); 0 means 2 */
    int32_t nz;       /* 0 or 1: a 2D mesh.  >= 2: a 3D mesh (nz, ny, nx), the extension
                         to three dimensions of Sec. 5 (periodic, even sides, order 2) */
    double dz;        /* mesh spacing along z (3D meshes); finite, > 0 */
} tsq_problem;

typedef struct tsq_plan tsq_plan; /* opaque, host memory */

/* Version of this ABI (TSQ_ABI_VERSION of the library that was loaded). */
int tsq_abi_version(void);

/* Message of the last failed call on the calling thread ("" if none).  The
 * pointer stays valid until the next tsq_* call on the same thread. */
const char* tsq_last_error(void);

/* Validate a problem and build a plan: the FP64 coefficients of the 2x2
 * block exponentials of the hopping parts H1 and H2 (Sec. 2: each block
 * [[0, V], [V, 0]], V = -hbar^2/(2 m a^2), exponentiates to a plane rotation
 * by al = tau |V| / hbar) for tau = dt/2 and dt along each axis, and a default
 * schedule.  Host only; touches no device.
 * Periodic 2D meshes apply the rotations in a tangent form (see
 * tsq_evolve) and accept |dt| hbar / (2 m da^2) < 1 rad per step along each
 * axis; closed 2D meshes apply it to the half-step even factors and accept
 * < 2 rad (larger steps are far outside the product's accuracy anyway).
 * Errors: TSQ_ERR_ARG (null, bad constant, order not 0/2/4), TSQ_ERR_SHAPE,
 * TSQ_ERR_DTYPE, TSQ_ERR_UNSUPPORTED (a 3D mesh with closed boundaries or
 * order 4; a 2D time step beyond that angle).  *out is set only on TSQ_OK. */
int tsq_plan_create(const tsq_problem* problem, tsq_plan** out);

/* Free a plan (NULL is accepted). */
int tsq_plan_destroy(tsq_plan* plan);

/* Bytes of device workspace the plan needs: a second psi buffer, the phase
 * table (complex128: one complex double per site; complex64: a hi/lo pair of
 * complex floats per site; order 4 keeps two tables, for the sub-steps of
 * p dt and (1-4p) dt) and reduction scratch.  Host only. */
int tsq_workspace_size(const tsq_plan* plan, size_t* bytes);

/* Schedule of the fused step kernel (2D meshes; a 3D mesh runs one step per
 * pass with its own tiling and takes only segment_rows, as the planes one
 * block marches).  Every schedule applies the same
 * operations in the same order to every site, so results are bitwise
 * identical across schedules; only speed changes. */
typedef struct {
    int32_t steps_per_pass;  /* time steps per read+write of psi in device memory:
                                1..8, 0 = default (5) */
    int32_t segment_rows;    /* rows marched by one wavefront: even, 0 = sized so one
                                launch is one round of resident wavefronts */
    int32_t pairs_per_lane;  /* x-pairs held by each lane: 1 or 2, 0 = default (1) */
    int32_t phase_store;     /* phase factors in flight: 1 = registers (steps_per_pass
                                <= 6, <= 4 with pairs_per_lane 2), 2 = LDS
                                (pairs_per_lane 1), 0 = default (registers up to 6
                                steps per pass, else LDS) */
} tsq_schedule;

/* Set the plan's schedule (host only).  Zero fields take their defaults;
 * tsq_plan_get_schedule returns the resolved values (segment_rows stays 0 when
 * it is sized per launch).  Errors: TSQ_ERR_ARG (null, value out of range, or
 * an unsupported combination: registers with more than 6 steps per pass, or
 * more than 4 with 2 pairs per lane; LDS with 2 pairs per lane; 2 pairs per
 * lane on a closed mesh); the plan keeps its previous schedule. */
int tsq_plan_set_schedule(tsq_plan* plan, const tsq_schedule* schedule);
int tsq_plan_get_schedule(const tsq_plan* plan, tsq_schedule* schedule);

/* Number of kernel launches (fused passes) tsq_evolve (or, after
 * tsq_set_potential_td, tsq_evolve_td) makes for `steps`
 * under the plan's schedule, and whether it ends with a device-to-device copy
 * (odd pass count that cannot be split).  Order-4 plans of periodic 2D meshes
 * run one pass per fourth-order step (its five second-order sub-steps fused,
 * whatever steps_per_pass says).  Host only.  Errors: TSQ_ERR_ARG. */
int tsq_evolve_passes(const tsq_plan* plan, int64_t steps, int64_t* passes, int32_t* copy_back);

/* The diagonal part H0 of Sec. 2 (potential plus the mesh's on-site term
 * eps_l = V_l + hbar^2/(m a^2) per axis) acts through exp(-i dt eps_l / hbar):
 * build that phase table exp(-i dt (V_l + eps0) / hbar) in FP64 from the device
 * array V_dev (nx*ny doubles) into the workspace `ws` of `ws_bytes` bytes
 * (device, 256-byte aligned).  On 2D meshes the table also carries the
 * cosines the tangent-form rotations leave out (see tsq_evolve).  complex128
 * stores it in FP64; complex64 as two int32 fixed-point parts scaled by 2^30
 * (8 bytes per site, about 31 bits each).
 * Records `ws`; tsq_evolve must be given the same workspace.
 * Errors: TSQ_ERR_ARG (null), TSQ_ERR_WORKSPACE, TSQ_ERR_DEVICE. */
int tsq_set_potential(tsq_plan* plan, const double* V_dev, void* ws, size_t ws_bytes,
                      void* stream);

/* Apply the second-order product U2(dt) of Eq. "secondorder" `steps` times
 * (order 4: U4(dt) of Eq. "fourthorder") to psi_dev in place (device,
 * contiguous, 16-byte aligned): several steps are fused per read and write of
 * psi (the schedule's steps_per_pass), consecutive odd factors merged.  On
 * periodic 2D meshes the even and odd-y factors rotate in the tangent form
 * (a, b) <- (a + i t b, b + i t a), t = tan al, and the phase factor and the
 * odd-x factors opening and closing the evolution restore the product of the
 * cosines; on closed 2D meshes the even factors rotate in the tangent form and
 * the phase factor restores their cosines site by site.  Equal to the block
 * exponentials in real arithmetic.  steps == 0 returns TSQ_OK without a launch.
 * Errors: TSQ_ERR_ARG (null, steps < 0, misaligned psi), TSQ_ERR_STATE (no
 * potential set, a different workspace, or a time-dependent table from
 * tsq_set_potential_td), TSQ_ERR_WORKSPACE, TSQ_ERR_DEVICE. */
int tsq_evolve(tsq_plan* plan, void* psi_dev, int64_t steps, void* ws, size_t ws_bytes,
               void* stream);

/* ---------------------------------------------------------------- time-dependent potential
 * V(t) = V0 + f(t) W.  The paper states the product for a time-independent
 * Hamiltonian and notes that the time-dependent form is the same construction
 * (Sec. 2, footnote to Eq. "evolution", citing Poulin et al.): here step n,
 * from t_n to t_n + dt, is U2(dt) with the potential frozen at the step's
 * midpoint, V0 + f_n W with f_n = f(t_n + dt/2), which keeps the product second
 * order for smooth f.  Order-2 plans of 2D meshes (periodic or closed); every step's phase factor
 * exp(-i dt (V0 + f_n W + eps0) / hbar) is formed in FP64 inside the march, so
 * up to 6 steps fuse per pass (a plan scheduled deeper runs 6). */

/* Store the time-dependent table of V0_dev and W_dev (device, nx*ny doubles
 * each) in `ws`: per site dt (V0 + eps0) / hbar and dt W / hbar (16 bytes, the
 * place of the phase table).  Records `ws` for tsq_evolve_td; a later
 * tsq_set_potential makes the workspace time-independent again.
 * Errors: TSQ_ERR_ARG (null), TSQ_ERR_UNSUPPORTED (order 4 or 3D mesh),
 * TSQ_ERR_WORKSPACE, TSQ_ERR_DEVICE. */
int tsq_set_potential_td(tsq_plan* plan, const double* V0_dev, const double* W_dev, void* ws,
                         size_t ws_bytes, void* stream);

/* Apply `steps` steps to psi_dev in place; step n uses f_host[n] (host array of
 * `steps` finite doubles, read before the call returns) as the modulation at
 * its midpoint.  Consecutive calls continue the evolution: pass each call the
 * modulations of its own steps.  Results are bitwise identical across
 * schedules.  Each step's phase angle dt (V0 + f_n W + eps0) / hbar must stay
 * below 2^42 in magnitude at every site (the in-kernel reduction's range; not
 * checked: larger angles give wrong phases).  Errors: TSQ_ERR_ARG (null,
 * steps < 0, a non-finite f, 2 pairs per lane, misaligned psi), TSQ_ERR_STATE
 * (tsq_set_potential_td not called with this workspace), TSQ_ERR_WORKSPACE,
 * TSQ_ERR_DEVICE. */
int tsq_evolve_td(tsq_plan* plan, void* psi_dev, int64_t steps, const double* f_host, void* ws,
                  size_t ws_bytes, void* stream);

/* FP64 norm N = sum |psi_l|^2, the quantity the unitary product conserves
 * (Sec. 2: |<psi|psi>| = 1), and energy E = <psi|H|psi> / N of the mesh
 * Hamiltonian of Sec. 2, H = diag(V + eps0) - Jx (x-neighbours) - Jy
 * (y-neighbours), J_a = hbar^2/(2 m da^2), neighbours wrapping periodically
 * (absent beyond closed walls).
 * Reduces in a fixed order (bitwise reproducible), uses the scratch part of
 * `ws` (it does not disturb the phase table), synchronises `stream` and
 * writes the two host doubles.  Errors: TSQ_ERR_ARG, TSQ_ERR_WORKSPACE,
 * TSQ_ERR_DEVICE. */
int tsq_observables(const tsq_plan* plan, const void* psi_dev, const double* V_dev,
                    double* norm_out, double* energy_out, void* ws, size_t ws_bytes,
                    void* stream);

/* ---------------------------------------------------------------- batched form
 * Many independent problems (each its own plan, psi, workspace and step
 * count; Sec. 2's problem statement per problem) advanced together: every
 * launch runs one pass of every problem that has one, as a fixed grid of
 * wavefronts walking a device work list of tiles sorted by height.  Results
 * are bitwise identical to tsq_evolve of each problem alone with the same
 * schedule. */
typedef struct tsq_batch tsq_batch; /* opaque, host memory */

/* Build a batch of n problems (host only): problem i is plans[i] applied to
 * psi_dev[i] with workspace ws[i] (tsq_set_potential must already have been
 * called with that workspace) for steps[i] >= 0 steps.  All plans must have
 * the same dtype and be periodic and of order 2, with a time-independent
 * potential on a 2D mesh (else TSQ_ERR_UNSUPPORTED).
 * `schedule` (NULL = defaults) applies to every problem; its segment_rows
 * is the height in rows of the batch's tiles (even; 0 = sized so one launch
 * is about one tile per resident wavefront).  The batch records the
 * device pointers, which must stay valid while it is used; plans may be
 * destroyed afterwards.  Errors: TSQ_ERR_ARG, TSQ_ERR_DTYPE (mixed dtypes),
 * TSQ_ERR_STATE (a plan without potential or with another workspace),
 * TSQ_ERR_DEVICE (device query failed). */
int tsq_batch_create(tsq_plan* const* plans, void* const* psi_dev, void* const* ws,
                     const int64_t* steps, int32_t n, const tsq_schedule* schedule,
                     tsq_batch** out);
int tsq_batch_destroy(tsq_batch* batch);

/* Device bytes of the batch's work lists (job records and tiles of every
 * launch), and the number of kernel launches and tiles one tsq_batch_launch
 * makes.  Host only. */
int tsq_batch_workspace_size(const tsq_batch* batch, size_t* bytes);
int tsq_batch_info(const tsq_batch* batch, int64_t* launches, int64_t* tiles);

/* Copy the work lists into `bws` (device, 256-byte aligned, at least
 * tsq_batch_workspace_size bytes), asynchronously on `stream`.  Must precede
 * tsq_batch_launch; `bws` must stay untouched while the batch is used.
 * Errors: TSQ_ERR_ARG, TSQ_ERR_WORKSPACE, TSQ_ERR_DEVICE. */
int tsq_batch_upload(tsq_batch* batch, void* bws, size_t bws_bytes, void* stream);

/* Enqueue every pass of every problem on `stream` (kernels and, for a
 * problem whose pass count is odd and cannot be split, one device copy).
 * With use_graph != 0 the sequence is captured into a HIP graph on the first
 * call (stream must not be the null stream) and replayed by later calls, on
 * any stream.
 * Each call advances every problem by its step count again.
 * Errors: TSQ_ERR_STATE (not uploaded), TSQ_ERR_ARG, TSQ_ERR_DEVICE. */
int tsq_batch_launch(tsq_batch* batch, int32_t use_graph, void* stream);

/* One call for the batched form: advance problem i (plans[i] on psi_dev[i]
 * with workspace ws[i], as for tsq_batch_create) by steps[i] steps, all
 * problems together, asynchronously on `stream`.  The work lists go to the
 * caller's device buffer `bws` of `bws_bytes` bytes (256-byte aligned, at least
 * what tsq_batch_evolve_workspace_size returns for the same arguments), which
 * must stay untouched until the work on `stream` has finished.  Equivalent to
 * tsq_batch_create + tsq_batch_upload + tsq_batch_launch (no graph) +
 * tsq_batch_destroy; results are bitwise identical to tsq_evolve of each
 * problem alone with the same schedule.  Errors: those of the four calls. */
int tsq_batch_evolve_workspace_size(tsq_plan* const* plans, void* const* psi_dev,
                                    void* const* ws, const int64_t* steps, int32_t n,
                                    const tsq_schedule* schedule, size_t* bytes);
int tsq_batch_evolve(tsq_plan* const* plans, void* const* psi_dev, void* const* ws,
                     const int64_t* steps, int32_t n, const tsq_schedule* schedule, void* bws,
                     size_t bws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * as tsq_batch_evolve, with the work lists in a device array the library holds
 * (16 MiB per GPU, kept until the process ends) instead of a caller buffer.
 * Allocates nothing.  Calls on one GPU share that array: calls that overlap
 * on one GPU (different streams, or host threads) race; calls in one stream
 * are ordered.  Errors: those of tsq_batch_evolve; TSQ_ERR_WORKSPACE when the
 * work lists (tsq_batch_evolve_workspace_size) exceed 16 MiB;
 * TSQ_ERR_DEVICE if the array's address cannot be found. */
int tsq_batch_evolve_noalloc(tsq_plan* const* plans, void* const* psi_dev, void* const* ws,
                             const int64_t* steps, int32_t n, const tsq_schedule* schedule,
                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TSQ_H */
