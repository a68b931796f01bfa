/*
 * lsr.h -- split-step round-trip map of a microchip-laser cavity on one
 * AMD Instinct MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * The method (Okulov, "Two-dimensional periodic and quasiperiodic spatial
 * structures in microchip laser resonator"): the intracavity field E(x,y)
 * on an N x N grid is carried bounce by bounce through the cavity map of the
 * Introduction, Eq. (1), in the form of Sec. 2.2, Eq. (11): a local step
 * (gain sheet whose inversion N(x,y) is frozen during the pass, mirror
 * reflectivity R, aperture D of Eq. (12)) followed by Fresnel diffraction over
 * the cavity length L, applied in Fourier space as the operator exponent
 * exp[i L/(2k) Laplacian] of Sec. 2.3, Eq. (25).  The inversion then relaxes
 * toward the pump and is depleted by |E|^2 (Eq. (1), second line, read as
 * the one-round-trip forward-Euler step of the B-class rate equation,
 * Eq. (6)).  One round trip n -> n+1, with sigma = 1:
 *
 *     I      = |E_n|^2
 *     G      = sqrt(R) A(x,y) exp(N_n/2) E_n            (local step)
 *     N_{n+1}= N_n + (N0(x,y) - N_n)/T1 - N_n I          (inversion update)
 *     E_{n+1}= IFFT2( H . FFT2(G) ),
 *              H = exp(-i pi lambda L (fx^2 + fy^2))     (diffraction)
 *
 * Grid: x_j = (j - N/2) dx, row-major (row y, column x) at index y*N + x;
 * fx = p~/(N dx) with the signed index p~ = p (p < N/2) else p - N.
 * Forward FFT unnormalized, inverse scaled by 1/N^2.
 *
 * Error behaviour: every entry point returns an lsr_status (0 = success);
 * nothing throws across the ABI.  lsr_last_error() gives a thread-local
 * message for the last failure on the calling thread.  GPU work is enqueued
 * asynchronously on the plan's stream: launch failures are reported by the
 * call, faults and non-finite state by the next synchronising call
 * (lsr_sync, lsr_diag, lsr_trace).
 *
 * Ownership: the caller owns E and Ninv (device memory, borrowed for the
 * duration of a call).  A plan owns its tables, scratch, trace ring and
 * graphs; a batch owns its task tables and counters but only borrows its
 * plans, which must outlive it.
 */
#ifndef LSR_H
#define LSR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsr_plan_s*  lsr_plan;
typedef struct lsr_batch_s* lsr_batch;

typedef enum {
    LSR_OK           =  0,
    LSR_EINVAL       = -1,   /* bad argument                                  */
    LSR_ENOMEM       = -2,   /* device or host allocation failed              */
    LSR_EDEVICE      = -3,   /* HIP runtime error (launch, copy, sync)        */
    LSR_EUNSUPPORTED = -4,   /* grid size or mode not compiled in             */
    LSR_ENONFINITE   = -5    /* the state became NaN/Inf (trip in message)    */
} lsr_status;

/* Arithmetic form of a plan.
 * PLAIN:     complex FP32 field and FFTs; twiddles generated in FP32
 *            arithmetic and the propagator phase pi lambda L (fx^2+fy^2)
 *            evaluated in FP32 on the device; diagnostics sums in FP64.
 * FP64TAB:   complex FP32 field and FFTs; twiddles and the propagator phase
 *            generated in FP64 and reduced modulo one turn before rounding
 *            to FP32; the propagator is the separable product hx(p) hx(q);
 *            diagnostics sums in FP64.
 * FP64:      the whole map in FP64 (validation form); E is complex128 and
 *            Ninv is double. */
typedef enum { LSR_PREC_PLAIN = 0, LSR_PREC_FP64TAB = 1, LSR_PREC_FP64 = 2 } lsr_prec;

/* Aperture modulus D0 of Eq. (12) (finite width of gain medium / mirror). */
typedef enum {
    LSR_AP_NONE = 0,         /* D0 = 1                                        */
    LSR_AP_SUPERGAUSS = 1,   /* D0 = exp(-(r/radius)^order), order even >= 2  */
    LSR_AP_GAUSS = 2,        /* D0 = exp(-r^2/(2 radius^2)), Eq. (26)         */
    LSR_AP_MASK = 3          /* D0 = mask[y*N + x]                             */
} lsr_aperture_kind;

typedef struct {
    int          kind;       /* lsr_aperture_kind                             */
    double       radius;     /* m                                             */
    int          order;      /* super-Gaussian exponent on r                  */
    const void*  mask;       /* kind 3: device float (double for FP64 plans)
                                N*N amplitude, borrowed for the plan's life   */
} lsr_aperture;

/* Diagnostics of one state (E_n, N_n), all sums taken in FP64:
 *   energy        W   = dx^2 sum |E|^2
 *   power_out     P   = (1-R) dx^2 sum |A|^2 e^N |E|^2  (leaves through the mirror)
 *   gain_sum          = dx^2 sum |A|^2 (e^N - 1) |E|^2  (added by the gain sheet)
 *   aperture_loss     = dx^2 sum (1 - |A|^2) |E|^2
 *   inv_sum           = dx^2 sum N
 * and the far-field radial spectrum of G = sqrt(R) A e^{N/2} E:
 *   radial[k] = sum over round(sqrt(p~^2 + q~^2)) = k of |FFT2(G)(p,q)|^2,
 *   k = 0 .. nbins-1, nbins = round(N/sqrt(2)) + 1;
 *   dominant_bin = argmax over k >= 1 (lowest on ties). */
typedef struct {
    double  energy, power_out, gain_sum, aperture_loss, inv_sum;
    int     dominant_bin;
    int     nbins;           /* out: number of bins of this plan               */
    double* radial;          /* in: host buffer of >= nbins doubles, or NULL   */
} lsr_diag_out;

/* Create a plan for one cavity.
 * N      grid points per side; supported: 256, 384, 512, 768, 1024, 2048, 4096
 *        (LSR_EUNSUPPORTED otherwise), in every precision form.
 * dx     grid spacing (m) > 0; lambda wavelength (m) > 0; L propagation length
 *        of one iterate (m) >= 0.  The Fresnel number is (N dx/2)^2/(lambda L).
 * F      mirror focal length (m) of the curvature phase exp(i k r^2/(2F)) of
 *        Eq. (12); 0 or +-INFINITY = flat mirror.
 * R      mirror reflectivity, 0 < R <= 1.
 * ap     aperture (NULL = LSR_AP_NONE).
 * The gain defaults to N0 = 0, T1 = 1 (set it with lsr_plan_set_gain), the
 * stream to the null stream.  Tables are built in FP64 on the host and
 * uploaded once; no allocation happens in later calls except lsr_diag's
 * first use of its spectrum scratch and table replacement by
 * lsr_plan_set_gain / lsr_plan_set_filter / lsr_plan_set_slices /
 * lsr_plan_set_roughness / lsr_propagate. */
int lsr_plan_create(lsr_plan* out, int N, double dx, double lambda, double L,
                    double F, double R, const lsr_aperture* ap, lsr_prec prec);

/* Local step and inversion update (sigma = 1, time in round trips, I the
 * intensity incident on the gain sheet, P the local pump level):
 * LSR_MODEL_B_EULER  (default) B-class laser, Eq. (1): amplitude gain
 *                    exp(N/2) with the inversion frozen during the pass, then
 *                    N' = N + (P - N)/T1 - N I (forward Euler over one trip).
 * LSR_MODEL_B_EXACT  the same gain; the rate equation of Eq. (6) integrated
 *                    exactly over one trip with I frozen:
 *                    N' = N_eq + (N - N_eq) exp(-(1/T1 + I)), N_eq = P/(1 + T1 I).
 * LSR_MODEL_CLASS_A  class-A laser, Eq. (8): saturable amplitude gain
 *                    exp(N / (2 (1 + T1 I))); the inversion state follows the
 *                    pump, N' = P.
 * The trace and diagnostics sums use the model's gain factor in place of
 * exp(N).  Takes effect on the next call, also in batches holding the plan
 * (a batch regroups its cavities when a model changes: a size whose
 * cavities all have one other model runs on kernels compiled for it, a size
 * with mixed models on kernels that read each cavity's model).
 * LSR_EINVAL for an unknown model. */
typedef enum { LSR_MODEL_B_EULER = 0, LSR_MODEL_B_EXACT = 1, LSR_MODEL_CLASS_A = 2 } lsr_model;
int lsr_plan_set_model(lsr_plan p, int model);

/* Free propagation of a field over a distance z (m), without the local step:
 * E_out = IFFT2( exp(-i pi lambda z (fx^2 + fy^2)) FFT2(E_in) ), the operator
 * exponent of Sec. 2.3, Eq. (25) for length z.  Used to record the field or
 * intensity at intermediate planes, e.g. the fractional Talbot planes of Sec. 5
 * (z = p^2 / (2 lambda m) for a pattern of period p).  E_in and E_out: device
 * N*N row-major complex fields of the plan's precision; they may be the same
 * buffer.  The phase table for z is built in FP64 and reduced mod one turn.
 * Asynchronous on the plan's stream; waits for that stream first and
 * allocates the table (the previous one is freed).  The plan's trace and
 * inversion are untouched.  LSR_EINVAL for z < 0 or non-finite. */
int lsr_propagate(lsr_plan p, const void* E_in, double z, void* E_out);

/* Nonlocal step of the map: delta > 0 replaces the Fresnel propagation by
 * the real renormalization-group filter of Sec. 2.3, Eq. (18),
 * exp[(delta^2/2) d^2/dx^2] applied along both transverse axes, i.e. the
 * Fourier multiplier exp(-2 pi^2 delta^2 (fx^2 + fy^2)); delta (m) is the
 * kernel's deviation.  delta = 0 restores the propagator.  The table is built
 * in FP64, as the propagator's; every precision form takes it from the table.
 * Waits for the plan's stream (the old table may still be in use) and
 * allocates the new table; batches holding the plan pick the change up on
 * their next call.  LSR_EINVAL for delta < 0 or non-finite. */
int lsr_plan_set_filter(lsr_plan p, double delta);

/* One-cavity FFT plan: k = 0 the size's default shape (the one batches use);
 * for N = 256 in the FP32 forms, k = 1 a shape with 8 points per lane and
 * twice the lanes per line (32 lanes x 8 lines, radices 8 8 4), k = 2 and 3
 * four points per lane (64 lanes, radix 4 throughout) on four and two lines
 * per workgroup; their shorter per-lane instruction chains suit a lone small
 * cavity.  For N = 2048 in the FP32 forms, k = 1 a wave per line (32 points
 * per lane), whose exchanges need no workgroup barrier.  Every plan computes the same transform
 * (results differ only by FP32 rounding); the twiddle table is rebuilt in
 * FP64 for the shape.  lsr_autotune(p, NULL, path) times the plans of the
 * size and keeps the fastest.  Waits for the plan's stream.  LSR_EUNSUPPORTED
 * where plan k is not compiled. */
int lsr_plan_set_fft_plan(lsr_plan p, int k);

/* General nonlocal step: the map with a kernel K of Eq. (10),
 * E_{n+1}(x2) = integral K(x1 - x2) G(x1) dx1 (Sec. 2.2; the real kernel of
 * the confocal 8F cavity, or any other convolution), given by its transfer
 * function: E_{n+1} = IFFT2(T . FFT2(G)).  T: HOST array of N*N complex
 * values (2*N*N doubles, interleaved re, im), frequency order, row-major
 * (row = y frequency index q, column = x frequency index p; index q*N + p);
 * read during the call only.  For a kernel sampled at the grid offsets u,
 * T(f) = dx^2 sum_u K(u) exp(+2 pi i f.u/N).  NULL restores the propagator
 * (or the filter of lsr_plan_set_filter).  The plan keeps T/N^2 by column in
 * its precision (8 B per point, 16 for FP64 plans), read by the column pass
 * in every precision form: the column pass then moves 8 (16) more bytes per
 * point.  One gain sheet only (LSR_EINVAL with several).  Batches run such
 * plans on the kernels that read each cavity's local-step code, whose column
 * tasks then take the cavity's table; setting or clearing T regroups a batch
 * holding the plan on its next call.  Waits for the plan's stream and
 * allocates the table (the previous one is freed).  LSR_EINVAL for a
 * non-finite value. */
int lsr_plan_set_transfer(lsr_plan p, const double* T);

/* Several thin gain sheets per round trip: the active medium spread along
 * the cavity instead of concentrated at one plane (the distributed-gain
 * variant the paper notes in Sec. 2.2 after Eq. (12)).  With m > 1 sheets a
 * round trip is m steps, k = 0..m-1: the local step of sheet k, then the
 * nonlocal step over L/m (propagator table built in FP64 for L/m; the filter
 * of lsr_plan_set_filter with variance delta^2/m, so that m steps make the
 * whole filter).  Sheet 0 carries the mirror (R, curvature) and the aperture
 * and holds the state E; the other sheets apply gain only.  Every sheet has
 * its own inversion, pump N0/m (the round trip's small-signal gain stays that
 * of one sheet), the plan's T1 and local-step model, and is depleted by the
 * field incident on it.  m = 1 (default) is the single sheet of Eq. (1).
 * After the call, lsr_roundtrips and lsr_time_kernels take Ninv as m*N*N
 * values, sheet k at element offset k*N*N; lsr_diag reads sheet 0; the trace
 * holds sheet 0's sums.  Launches: 2m per trip plus 1.  Waits for the plan's
 * stream and allocates the table of the step (the previous one is freed).
 * Batches run plans of any sheet counts together: the plans of one count
 * form groups whose sheet step k is one grouped row pass and one grouped
 * column pass over their cavities (or one persistent launch), and step k
 * launches the groups with more than k sheets; a changed count regroups the
 * batch on its next call.
 * LSR_EINVAL unless 1 <= m <= LSR_MAX_SLICES. */
#define LSR_MAX_SLICES 64
int lsr_plan_set_slices(lsr_plan p, int m);

/* Mirror roughness: the random phase psi(x, y) of the complex aperture of
 * Sec. 2.2, Eq. (12), D = D0 exp(i k r^2/(2F) + i psi), on top of the
 * curvature phase of F.  psi: HOST array of N*N doubles (rad), row-major
 * (element (row y, column x) at y*N + x), read during the call only; NULL
 * restores the smooth mirror.  The plan builds exp(i psi) in FP64 (each angle
 * reduced to one turn first), keeps it in device memory in its precision
 * (8 B per point, 16 for FP64 plans) and applies it in the local step at the
 * mirror sheet: the row pass then reads that many more bytes per point.
 * Rough plans run on kernels compiled with the roughness factor (the default
 * kernels carry none); a batch holding the plan regroups on its next call
 * (sizes with a rough cavity run on kernels that read each cavity's code),
 * as after a model change.  Waits for the plan's stream and allocates the
 * table (the previous one is freed).  Diagnostics (lsr_diag) include it.
 * LSR_EINVAL for a non-finite psi. */
int lsr_plan_set_roughness(lsr_plan p, const double* psi);

/* Pump and relaxation (Eq. (1), second line; periodic pump of Sec. 3):
 * N0(x,y) = N0 (1 + mod_amp cos(2 pi x/mod_period) cos(2 pi y/mod_period)),
 * uniform when mod_amp = 0 or mod_period = 0.  T1 > 0 in round trips. */
int lsr_plan_set_gain(lsr_plan p, double N0, double T1, double mod_amp,
                      double mod_period);

/* Bind the plan to a HIP stream (hipStream_t passed as void*; NULL = null
 * stream).  All later work of the plan is enqueued on it. */
int lsr_plan_set_stream(lsr_plan p, void* hip_stream);

/* Advance the state n_trips >= 0 round trips, in place, asynchronously.
 * E    device complex64 (complex128 for FP64 plans) N*N, row-major, the field
 *      at the gain sheet before the local step (E_n in, E_{n+n_trips} out).
 * Ninv device float (double for FP64 plans) N*N, row-major (N_n in, out);
 *      m*N*N (one map per sheet) after lsr_plan_set_slices(p, m).
 * Both must be 16-byte aligned and must not overlap.  During the call E's
 * memory also holds the transformed field in an internal tiled layout; it is
 * row-major again when the enqueued work completes.  Launches: 2 per trip
 * plus 1.  The per-trip diagnostics sums go to the plan's trace ring. */
int lsr_roundtrips(lsr_plan p, void* E, void* Ninv, int n_trips);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the round
 * trips of lsr_roundtrips in the FP64TAB form without a plan, and without any
 * allocation.  The arguments are those of lsr_plan_create (N, dx, lambda, L,
 * F, R, ap), lsr_plan_set_gain (N0, T1, mod_amp, mod_period) and
 * lsr_plan_set_model (model), then E (device complex64 N*N) and Ninv (device
 * float N*N) as for lsr_roundtrips, n_trips >= 0, trace (device, 4*n_trips
 * doubles receiving each trip's S1..S4 as lsr_trace returns them, or NULL)
 * and the stream (hipStream_t as void*, NULL = null stream).
 * The FP64-built tables, the per-row-block partial sums and the counters live
 * in a file-scope device array of 512 KiB that each GPU holds until the
 * process ends; a small kernel rebuilds the tables and clears the counters at
 * the start of every call, then the call enqueues the launches of
 * lsr_roundtrips (kernel launches only: no allocation, copy, memset or
 * synchronisation).  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (on different streams, or from several threads)
 * race and give wrong results.  No mirror roughness and one gain sheet; the
 * non-finite state is not reported (the trace shows it).  LSR_EINVAL for bad
 * arguments or a size whose tables exceed the array, LSR_EUNSUPPORTED for N
 * not compiled in. */
int lsr_roundtrips_static(int N, double dx, double lambda, double L, double F, double R,
                          const lsr_aperture* ap, double N0, double T1, double mod_amp, double mod_period,
                          int model, void* E, void* Ninv, int n_trips, double* trace, void* stream);

/* Wait for the plan's stream; LSR_ENONFINITE if any trip since the last
 * lsr_sync saw a non-finite state (the flag is cleared by the report). */
int lsr_sync(lsr_plan p);

/* Copy the raw per-trip sums of the last lsr_roundtrips call (oldest first)
 * to host memory: out[4t+0..3] = S1 = sum|E|^2, S2 = sum|A|^2|E|^2,
 * S3 = sum|A|^2 e^N |E|^2, S4 = sum N of the incoming state of trip t.
 * Copies min(capacity, n_trips of that call, ring size) records; returns the
 * count (>= 0) or a negative status.  Synchronises the stream. */
int lsr_trace(lsr_plan p, double* out, int capacity);

/* Profiling form of lsr_roundtrips: the same launches, each bracketed by
 * HIP events on the plan's stream.  Writes the mean duration in ms of the
 * row-pass kernel (ms[0]) and the column-pass kernel (ms[1]) over the
 * n_trips >= 1 trips; synchronises. */
int lsr_time_kernels(lsr_plan p, void* E, void* Ninv, int n_trips, double* ms);

/* Diagnostics of the state (E, Ninv), the quantities of lsr_diag_out: the
 * power leaving through the output mirror, the plane whose transverse
 * patterns the paper models (abstract), with the gain and aperture balance
 * of the local step of Eq. (1) and Eq. (12); and the far-field spectrum of
 * the field leaving the gain sheet, in the spirit of the Fourier images of
 * Sec. 5, whose dominant transverse wavevector gives the pattern period.  E and Ninv as for
 * lsr_roundtrips (read only).  Uses the plan's spectrum scratch (allocated
 * on the first call); synchronises the stream.  LSR_ENONFINITE if the sums
 * are not finite. */
int lsr_diag(lsr_plan p, const void* E, const void* Ninv, lsr_diag_out* out);

/* Number of radial spectrum bins of a plan (round(N/sqrt(2)) + 1). */
int lsr_plan_nbins(lsr_plan p);

void lsr_plan_destroy(lsr_plan p);

/* ---------------------------------------------------------------------- */
/* Batching: many cavities of uneven N and parameters advanced together,  */
/* by one grouped launch per pass or one persistent kernel per round trip, */
/* replayed as HIP graphs.  Batches take LSR_PREC_FP64TAB plans, any       */
/* local-step model, roughness and filter, and one number of gain sheets.  */
/* ---------------------------------------------------------------------- */

/* Build a batch over count >= 1 plans (borrowed: they must outlive the
 * batch and are not copied): many independent cavities, of any mix of the
 * supported sizes and parameters, advanced together by the map of Intro
 * Eq. (1) with the nonlocal step of Sec. 2.2 (Eqs. (11)-(12)).  The launch
 * configuration (FFT plan, engine, register budget, grouping, task-table
 * lag, graph length k) comes from the autotune cache when it holds an entry
 * for this mix of sizes, else from built-in defaults.  The batch runs on
 * the stream its plans are bound to: every plan must be bound to the same
 * stream (LSR_EINVAL otherwise, here and in every later call that finds a
 * plan rebound to another one).  Errors: LSR_EINVAL for a NULL out or plan,
 * count < 1, a plan given twice or plans on different devices;
 * LSR_EUNSUPPORTED for plans other than the FP64TAB form; LSR_ENOMEM /
 * LSR_EDEVICE when its tables or task lists cannot be allocated or uploaded
 * (nothing is leaked; *out is then NULL). */
int lsr_batch_create(lsr_batch* out, const lsr_plan* plans, int count);

/* Advance cavity i's state (E[i], Ninv[i]: device buffers laid out as for
 * lsr_roundtrips, owned by the caller, borrowed for the call) by n_trips >= 0
 * round trips of the map of Intro Eq. (1), all cavities together,
 * asynchronously on the plans' stream; the results equal lsr_roundtrips on
 * each plan bit for bit with the default FFT plans.  The per-trip sums go to
 * each plan's trace ring.  E and Ninv hold one pointer per plan, in the
 * order of lsr_batch_create.  Errors: LSR_EINVAL for a NULL batch, array or
 * state pointer, a pointer not 16-byte aligned, n_trips < 0 or a plan bound
 * to another stream; LSR_ENOMEM when a plan's changed local step, nonlocal
 * step or number of gain sheets needs a regrouping that cannot allocate;
 * LSR_EDEVICE when a launch fails.  A non-finite state is reported by
 * lsr_sync of its plan. */
int lsr_batch_roundtrips(lsr_batch b, void* const* E, void* const* Ninv, int n_trips);

/* Diagnostics of cavity idx of the batch; same as lsr_diag on its plan. */
int lsr_batch_diag(lsr_batch b, int idx, const void* E, const void* Ninv,
                   lsr_diag_out* out);

/* Set the trips per captured graph (k >= 1; 0 = no graph, eager launches). */
int lsr_batch_set_graph_trips(lsr_batch b, int k);

/* Capture and instantiate, without running anything, the HIP graphs that a
 * later lsr_batch_roundtrips call of n_trips >= 0 trips replays, so that the
 * capture cost is not paid inside that call.  With graph length k > 0 a call
 * of n <= k + 1 trips replays one graph of the whole call (first row pass,
 * n - 1 middle trips, last row pass); a longer call runs its first and last
 * row passes as launches around (n - 1)/k graphs of k middle trips and one
 * graph of the (n - 1) mod k remaining ones.  A batch keeps up to 8 graphs
 * and drops the least recently used one (after the stream has drained) when
 * it needs another; regrouping, repacking or reconfiguring drops them all.
 * Graphs read the descriptors and task tables from device memory, so new
 * state pointers or plan parameters need no new capture. */
int lsr_batch_prepare(lsr_batch b, int n_trips);

/* Failure-path hook for tests of the persistent engine (engine 0): the
 * column tasks' bounded wait for their cavity's row blocks polls at most
 * spin_limit times (0 = about 2 s) and waits for extra_need more row blocks
 * than exist (0 = the real count).  With extra_need > 0 every wait gives up,
 * every cavity is flagged and its column tasks are skipped; the kernels still
 * run to completion, and lsr_sync of each plan reports LSR_EDEVICE.  Both
 * values return to 0 when the batch regroups.  Synchronises. */
int lsr_batch_test_wait(lsr_batch b, int extra_need, int spin_limit);

/* Launch configuration of a batch; a negative argument keeps the current
 * value.  engine: 0 = one persistent kernel per round trip (task queue with
 * per-cavity row-to-column dependencies), 1 = one grouped launch per pass
 * (every cavity's row blocks, then every cavity's column blocks), 2 = grouped
 * launches whose resident workgroups prefetch their next task's data while
 * computing the current one (groups of a single grid size; other groups fall
 * back to 1).  variant:
 * register budget of the kernels: 0 = four waves per SIMD (128 VGPRs; a
 * kernel that needs more spills a few registers), 1 = two waves per SIMD
 * (256); 4096 and the mixed-size kernels have one budget.
 * wgs_per_cu: resident workgroups per CU of the persistent kernel (0 =
 * occupancy limit).  chunk: tickets taken per queue access.  lag: packer lag
 * in row tasks.  graph_k: trips per captured graph (0 = eager).  merge:
 * 0 = one kernel per grid size (each specialised for its size), 1 = cavities
 * of uneven grid sizes with the same workgroup size share one kernel (one
 * persistent launch per trip covers them all).  shape: FFT plan of the
 * one-size groups (merge = 0): 0 = each size's default plan (the one-cavity
 * path's), k = 1 .. LSR_MAX_SHAPES = alternative plan k of the sizes that
 * have one compiled (others keep their default):
 *   1  reversed radix order: 512 as 16 8 4, 1024 as 16 16 4, 2048 as 16 16 8;
 *      4096 with 128 lanes per line (32 points per lane, 512 threads);
 *      256 with 8 points per lane (the one-cavity FFT plan 1 of that size);
 *   2  1024 on 8 x 8 tiles, eight lines per workgroup.
 * Every plan computes the same transform; with an alternative plan the
 * batch's results differ from the one-cavity path's only by rounding (they
 * are bitwise equal with shape 0).  cfg_out (nullable) receives the
 * resulting eight values in this order. */
#define LSR_MAX_SHAPES 2
int lsr_batch_configure(lsr_batch b, int engine, int variant, int wgs_per_cu, int chunk,
                        int lag, int graph_k, int merge, int shape, int* cfg_out);

/* Profiling form of lsr_batch_roundtrips (eager, no graph): each pass is
 * launched with HIP events that the dispatch itself timestamps at kernel
 * start and end (hipExtLaunchKernelGGL), on the batch's stream.  ms[0] =
 * mean duration of the row-pass launch (all cavities' row blocks of one
 * trip, middle trips only when n_trips > 1), ms[1] = mean column-pass
 * launch, ms[2] = mean round trip from one row-pass start to the next
 * (ms[0] + ms[1] + the gaps between them).  With several gain sheets ms[0]
 * and ms[1] sum the row and column passes of a trip's sheet steps.  With
 * the persistent engine the whole trip is one launch per sheet step:
 * ms[0] = ms[2], ms[1] = 0.  Synchronises. */
int lsr_batch_time_kernels(lsr_batch b, void* const* E, void* const* Ninv, int n_trips, double* ms);

void lsr_batch_destroy(lsr_batch b);

/* Autotune: time the candidate configurations of batch b (lsr_batch_configure:
 * FFT plan, engine, register budget, grouping, persistent-kernel chunk, lag
 * and residency, graph length) on the device with scratch state, keep the
 * fastest, and store it in the JSON cache at cache_path (NULL =
 * $LSR_TUNE_CACHE or no file).  The winner applies to the batch at once and
 * to later batches of the same sizes.  A plan alone (b = NULL): the cached
 * one-cavity FFT plan of its size and precision form if the cache holds one,
 * else the fastest of its compiled one-cavity FFT plans, timed on scratch
 * state and stored; applied to the plan (lsr_plan_set_fft_plan).
 * Synchronises. */
int lsr_autotune(lsr_plan p, lsr_batch b, const char* cache_path);

/* ---------------------------------------------------------------------- */
/* Host-side introspection (no GPU needed).                                 */
/* ---------------------------------------------------------------------- */

const char* lsr_last_error(void);
const char* lsr_version(void);

/* Failure-path hook for tests: the device allocation made after `after`
 * more successful ones (0 = the next one) fails as if the device were out of
 * memory, once; -1 switches the hook off.  Every entry point that allocates
 * then returns LSR_ENOMEM and frees what it had allocated in that call. */
int lsr_test_fail_alloc(int after);

/* Whether grid size N is compiled in for prec (1) or not (0). */
int lsr_supported(int N, int prec);

/* The FFT factorisation used for N: writes up to max radices (forward pass
 * order) to radices and returns their count, lanes per line and lines per
 * workgroup; negative status if N is unsupported. */
int lsr_fft_shape(int N, int prec, int* radices, int max, int* lanes_per_line,
                  int* lines_per_group);

/* The FP64-built per-axis propagator table of an FP64TAB plan:
 * out[2p], out[2p+1] = Re, Im of hx(p) = exp(-i pi lambda L fx_p^2) / N,
 * the phase reduced modulo one turn in FP64 before rounding; p = 0..N-1.
 * Pure host arithmetic, for inspection and tests. */
int lsr_propagator_table(int N, double dx, double lambda, double L, float* out);

/* The Stockham twiddle tables of grid size N (forward then inverse passes,
 * concatenated; per pass with sub-length Ns > 1 and radix R, Ns*R entries
 * w(k, r) = exp(-+2 pi i r k/(Ns R)), k < Ns, r < R), as interleaved floats
 * built in FP64 (prec FP64TAB and FP64; the FP64 shape's passes for FP64) or
 * in FP32 arithmetic (PLAIN), returned rounded to float.  Layout inside a
 * segment, for the lanes of a wave to read contiguous memory: for the FP32
 * forms and even R, w(k, r) sits at (r/2)*2*Ns + 2k + r%2 (the pair r, r+1
 * of one k adjacent); for odd R, and for FP64, at r*Ns + k.  Returns the number of complex entries, or the
 * required count if out is NULL. */
int lsr_twiddle_table(int N, int prec, float* out, int capacity);

/* The batch packer's task order for a set of grid sizes, host only:
 * writes per task (cavity index, kind 0 = row block / 1 = column block,
 * block index) triples to tasks (3 ints each) and returns the task count;
 * with tasks = NULL returns the count only.  The column tasks of a cavity
 * follow once lag further row tasks have been issued after its last row task
 * (-1 = default 2048).  Every column task's row tasks come before it. */
int lsr_pack_tasks(const int* sizes, int count, int lag, int* tasks, int capacity);

#ifdef __cplusplus
}
#endif
#endif /* LSR_H */
