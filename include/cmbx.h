/*
 * cmbx -- partial-sky CMB maps from a periodic 3-D box (MI355X / gfx950).
 *
 * Method: Giner Mascarell & Bunn, "Simulating Partial Sky Cosmic Microwave Background
 * Maps with 3D Fast Fourier Transforms" (arXiv:2507.15703), Sec. II D 1 (the 3-D Fourier
 * method): fill the box's Fourier modes with complex normals of variance P_box(|k|),
 * inverse-FFT to a real field, and interpolate the field at the sky pixels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Box: N^3 nodes, side L, node j at j L / N, periodic. N must be even, 8 <= N <= 1024,
 *   and of the form 2^a 3^b with N/2 also of that form.
 * - Observer at the box centre c = (L/2, L/2, L/2) unless cmbx_plan_observer moves it;
 *   pixel with unit direction n sits at c + r n. In grid units p = (r n + c) (N / L),
 *   evaluated in FP64; the stencil is chosen by floor(p) and node indices wrap modulo N.
 * - Spectrum normalisation: the caller gives P_inf(k), the infinite-space spectrum with
 *   xi(r) = int d^3k P_inf e^{i k.r} (Sec. II A, eq. xiinfpinf); the box uses
 *   P_box = P_inf (2 pi / L)^3 (Sec. II C, eq. finalpbox with M = N) and drops k = 0.
 * - Noise: mode (ix, iy, iz) of the half grid (iz = 0 .. N/2) is driven by Philox4x32-10
 *   with key = (seed & 0xffffffff, seed >> 32) and counter (iz >> 1, iy, ix, 0), words
 *   (x0, x1) for even iz and (x2, x3) for odd iz, through a fixed-operation FP64
 *   Box-Muller transform; generic modes get sqrt(P_box/2) (g_re + i g_im), the planes
 *   iz = 0, N/2 are made Hermitian, and the 8 self-conjugate modes are sqrt(P_box) g_re.
 *   Realisation b of a batch uses seed + b.
 * - Inverse DFT: unnormalised, + sign: T(j) = sum_f T(f) exp(+2 pi i f.j / N).
 * - All device pointers are HIP device memory owned by the caller unless stated. Calls
 *   that launch work are asynchronous on the plan's stream; the caller synchronises.
 * - Every function returns CMBX_OK (0) or a negative error code and never throws;
 *   cmbx_last_error() gives the message of the calling thread's last failure.
 */
#ifndef CMBX_H
#define CMBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CMBX_OK            0
#define CMBX_EINVAL       -1  /* an argument is out of range or NULL */
#define CMBX_EUNSUPPORTED -2  /* a valid request this build does not implement (e.g. N = 2^a 3^b 5^c) */
#define CMBX_ENOMEM       -3  /* a device or host allocation failed */
#define CMBX_EHIP         -4  /* a HIP runtime call failed (no device, launch error) */
#define CMBX_ESTATE       -5  /* call out of order (e.g. simulate before a spectrum is set) */
/* Tests of the error paths can make some sites fail as the runtime would: the environment
 * variable CMBX_FAULT, read at each call, holds a comma-separated list of "alloc" (plan
 * allocation: CMBX_ENOMEM), "capture" (ensemble graph capture: CMBX_EHIP) and "launch"
 * (ensemble launch: CMBX_EHIP). Unset, it costs one getenv per such call. */

/* working precision of a plan */
#define CMBX_F32 1
#define CMBX_F64 2

/* interpolants (option CMBX_OPT_INTERP) */
#define CMBX_TRILINEAR 1 /* 2 nodes per axis, K(x) = 1 - |x| */
#define CMBX_TRICUBIC  2 /* 4 nodes per axis, Keys cubic convolution with a = -1/2 */

/* plan options for cmbx_plan_set */
#define CMBX_OPT_INTERP   1 /* CMBX_TRILINEAR (default) or CMBX_TRICUBIC */
#define CMBX_OPT_STREAM   2 /* hipStream_t cast to int64_t (0 = the null stream); -1 = the plan's own stream (default) */
#define CMBX_OPT_TILE_XY  3 /* columns per workgroup of both the x and y passes; 0 = default */
#define CMBX_OPT_LINES_Z  4 /* lines per workgroup of the z pass; 0 = default */
#define CMBX_OPT_TILE_X   5 /* columns per workgroup of the x pass (noise + x transform) */
#define CMBX_OPT_TILE_Y   6 /* columns per workgroup of the y pass */
/* 1 (default): maps are made from only the part of the field their pixels' interpolation
 * stencils read (the map footprint, found on the device from the directions at every
 * call); 0: from the whole field. The maps are the same either way (Sec. II D 1: the box
 * is simulated and then sampled; only the samples are the product). */
#define CMBX_OPT_PRUNE    7
/* 1: the caller keeps the directions at a given address unchanged (the paper's batches of
 * maps of one cap, Sec. IV). A pruning plan then makes the map footprint once per
 * (r, dirs, n_pix, interpolant, z tile, observer) and reuses it in later
 * cmbx_simulate_patch calls, and an ensemble created from it makes its footprints once at
 * creation instead of inside its graph at every launch. Any plan with the option also
 * sorts the pixels once per (r, dirs, n_pix, interpolant, observer) by the Morton code of
 * their stencils' first node and gathers in that order (neighbouring threads read the same
 * field lines; each pixel's value is the same bit for bit, and out keeps the caller's
 * order): cmbx_simulate_patch and cmbx_time_passes keep the order in the plan (not made
 * while the plan's stream is being captured: the gather then reads the directions), an
 * ensemble makes one per realisation at creation for its chained gathers. Setting the
 * option (again, to 0 or 1) drops the kept footprint and order: do so after writing new
 * directions at the same address. Default 0: the footprint is made from the directions at
 * every call and the gather reads them in the caller's order. */
#define CMBX_OPT_FIXED_DIRS 8
/* FFT stage plan of the x, y and z pass: 0 (default) or 1, an alternative factorisation of
 * the transform length into radix stages (e.g. 512 = 16 x 8 x 4 instead of 8 x 8 x 8,
 * 256 = 4 x 8 x 8 instead of 16 x 16), compiled for lengths with a power-of-two part of at
 * least 32 and for the pass's default tile only: setting plan 1 sets that tile, and
 * setting another tile sets plan 0. cmbx_plan_autotune chooses among them. */
#define CMBX_OPT_PLAN_X   9
#define CMBX_OPT_PLAN_Y   10
#define CMBX_OPT_PLAN_Z   11

typedef struct cmbx_plan cmbx_plan;
typedef struct cmbx_ensemble cmbx_ensemble;

/*
 * Create a plan for a batch of `batch` realisations of an N^3 box of side L in precision
 * `dtype`. The plan owns its device workspace (batch x N^3 reals: the field, computed in
 * place), the twiddle table and the weight table, on the device current at the call.
 * Errors: CMBX_EINVAL (out == NULL, N odd or < 8 or > 1024, L <= 0 or not finite,
 * batch < 1, unknown dtype), CMBX_EUNSUPPORTED (N not 2^a 3^b), CMBX_EHIP (no device),
 * CMBX_ENOMEM. On error *out is set to NULL.
 */
int cmbx_plan_box(int N, double L, int dtype, int batch, cmbx_plan** out);

/* Release a plan and its device memory (waits for its stream). NULL is accepted. */
int cmbx_plan_destroy(cmbx_plan* plan);

/* Observer position o = (x, y, z) in the box, in the units of L (default: the centre,
 * L/2 each). Pixels then sit at o + r n: in grid units p = (r n + o) (N / L), in FP64 and
 * in that order, every later gather, map and footprint of the plan (an ensemble keeps the
 * position its plan had at creation). Sec. II D 1 places the box about the cap rather than
 * about the observer: with the cap about +z at radius r, the box centre on the cap's axis
 * at height r (1 + z_min) / 2 is the observer at (L/2, L/2, L/2 - r (1 + z_min) / 2); any
 * position is reduced modulo the periodic box. CMBX_EINVAL for a non-finite coordinate. */
int cmbx_plan_observer(cmbx_plan* plan, double x, double y, double z);
/* The observer that places the plan's box about a cap (Sec. II D 1, Fig. 2a): the cap about
 * +z at radius r > 0 with edge z_min = cos(theta_max) in [-1, 1], the box centre on its
 * axis at height r (1 + z_min) / 2, i.e. xyz = (L/2, L/2, L/2 - r (1 + z_min) / 2). Writes
 * the three coordinates to xyz (host) and changes nothing (pass them to cmbx_plan_observer).
 * CMBX_EINVAL for a bad r, z_min or NULL xyz. */
int cmbx_plan_cap_observer(const cmbx_plan* plan, double r, double z_min, double* xyz);

/* Set a plan option (CMBX_OPT_*). CMBX_EINVAL for an unknown key or a bad value. */
int cmbx_plan_set(cmbx_plan* plan, int key, int64_t value);

/* Read an option back (CMBX_OPT_INTERP, _TILE_X, _TILE_Y, _LINES_Z (the tiles in use, the
 * defaults resolved), _PRUNE, _FIXED_DIRS, _PLAN_X/Y/Z) into *value. CMBX_EINVAL for a NULL
 * plan or value or another key. */
int cmbx_plan_get(const cmbx_plan* plan, int key, int64_t* value);

/* Read back a plan's geometry: any output pointer may be NULL. */
int cmbx_plan_info(const cmbx_plan* plan, int* N, double* L, int* dtype, int* batch,
                   void** field);

/*
 * Set the plan's spectrum from a host table of P_inf(k) (Sec. II B-C). k (strictly
 * increasing, >= 0) and P_inf (>= 0, finite) are host FP64 arrays of length n >= 2,
 * copied; P_inf is linear in k between nodes and zero outside [k[0], k[n-1]] (the
 * cut-off beyond which the spectrum is taken to vanish, Sec. II B). The per-|k|^2 weight
 * table sqrt(P_box/2) is formed in FP64 on the host, rounded once to the plan's
 * precision and uploaded. Errors: CMBX_EINVAL, CMBX_ENOMEM, CMBX_EHIP.
 */
int cmbx_spectrum_table(cmbx_plan* plan, const double* k, const double* P_inf, int64_t n);

/*
 * Simulate the plan's batch and sample it on a sky patch (Sec. II D 1).
 *   seed   realisation b uses seed + b
 *   r      shell radius, 0 < r < L/2 (observer at the centre; once cmbx_plan_observer has
 *          moved it, any finite r > 0: keeping the cap inside the box is the caller's part)
 *   dirs   device FP64 [n_pix][3] unit vectors (caller-owned)
 *   out    device array [batch][n_pix] of the plan's precision (caller-owned)
 * The field of realisation b is left in the plan's workspace (cmbx_plan_info): the whole
 * field with CMBX_OPT_PRUNE 0, otherwise only the z-lines in 8-row blocks of x-planes
 * that the pixels' stencils read (the rest of the workspace is left as it was).
 * Errors: CMBX_ESTATE (no spectrum yet), CMBX_EINVAL (r out of range, n_pix < 1, NULL
 * pointer), CMBX_EHIP (launch failure).
 */
int cmbx_simulate_patch(cmbx_plan* plan, uint64_t seed, double r, const double* dirs,
                        int64_t n_pix, void* out);

/* ---- ensembles: many jobs of mixed box sizes per launch sequence ---- */

typedef struct cmbx_job {
  cmbx_plan* plan;     /* plan of this job (its batch is simulated; its workspace is used) */
  uint64_t seed;       /* as cmbx_simulate_patch */
  double r;
  const double* dirs;  /* device [n_pix][3] */
  int64_t n_pix;
  void* out;           /* device [batch][n_pix] */
} cmbx_job;

/* ensemble execution modes */
#define CMBX_ENS_AUTO      0 /* time the modes and lanes at creation, keep the fastest */
#define CMBX_ENS_CHAINED   1 /* each realisation's four kernels in turn, in its plan's workspace */
#define CMBX_ENS_PIPELINED 2 /* software pipeline of fused launches (see below) */
/* lane flags, OR-ed into the mode */
#define CMBX_ENS_LANES(n)  ((n) << 8) /* chained items split by plan over n graphs (1 <= n <= 4) */
#define CMBX_ENS_ONE_LANE  CMBX_ENS_LANES(1) /* one graph on the launch stream */
#define CMBX_ENS_TWO_LANES CMBX_ENS_LANES(2) /* two graphs on two streams */
#define CMBX_ENS_MAX_LANES 4

/*
 * Capture the jobs into one HIP graph. Every realisation of every job (job j's plan has
 * `batch` of them, seeds seed + b, maps at out + b n_pix) is an item; items of equal
 * (precision, N) form a group, and groups run one after another in job order.
 * - CMBX_ENS_CHAINED: the items of a group run one after another, each through the same
 *   four kernels (tile shapes as set on its plan) in its plan's workspace slot b.
 * - CMBX_ENS_PIPELINED: launch t of a group runs, side by side in one kernel, the noise + x
 *   pass of item t, the y pass of item t-1, the z pass of item t-2 and the gather of item
 *   t-3 (workgroups of the four roles interleaved), on min(4, items) workspaces owned by
 *   the ensemble.
 * - CMBX_ENS_AUTO: both are captured for each group and timed (the outputs are written
 *   meanwhile); the faster is kept (cmbx_ensemble_modes reports the choice).
 * Lanes: with CMBX_ENS_LANES(n) the chained items are split by plan (all items of one plan
 * in one lane, since they share its workspace; heaviest plans first into the lightest
 * lane) into n graphs. Lane 0 (with every pipelined group) runs on the launch stream,
 * lanes 1 .. n-1 on streams the ensemble owns, forked from and joined back into the launch
 * stream, so the chains of different plans can overlap on the device. There are never
 * more lanes than chained plans. Without a lane flag, CMBX_ENS_AUTO times the whole
 * ensemble with the per-group choice and with every group chained, on each possible
 * number of lanes up to CMBX_ENS_MAX_LANES (each candidate scored by the median of six
 * timings taken in alternating sweeps), and keeps the fastest, or among those within
 * 1 % of it the one with the fewest lanes, two counting before one where two are possible
 * (so it may report a group chained that was
 * faster pipelined alone); the explicit modes use one lane. Launches of one ensemble must be
 * ordered (one launch stream, or synchronised).
 * Buffers passed in stay caller-owned and must outlive the ensemble, and so must the
 * plans, whose weight and twiddle tables and workspaces are used when the graph runs
 * (interpolant, prune option, r and pixel counts are fixed at creation; a pruning plan's
 * footprint is made from the directions at every launch, or once at creation if the plan
 * has CMBX_OPT_FIXED_DIRS). Errors: as cmbx_simulate_patch
 * for each job, CMBX_EINVAL for n_jobs < 1, an unknown mode or more than
 * CMBX_ENS_MAX_LANES lanes,
 * CMBX_ENOMEM.
 */
int cmbx_ensemble_create(const cmbx_job* jobs, int n_jobs, int mode, cmbx_ensemble** out);
/* Number of lanes (1 .. CMBX_ENS_MAX_LANES) the ensemble runs in, or CMBX_EINVAL for a
 * NULL ensemble. */
int cmbx_ensemble_lanes(const cmbx_ensemble* ens);
/* Mode chosen for each group (in order of first appearance) written to modes[0 .. cap);
 * returns the number of groups, or CMBX_EINVAL for a NULL ensemble. */
int cmbx_ensemble_modes(const cmbx_ensemble* ens, int* modes, int cap);
/* Launch the captured graphs on `stream` (a hipStream_t; NULL = the default stream): the
 * work is ordered after what `stream` already holds, and what is later enqueued on
 * `stream` runs after all of it. The captured kernels skip the modes beyond each plan's
 * spectral support (the largest |f|^2 of nonzero weight) as it was at creation: a plan's
 * table may change between launches, but CMBX_ESTATE is returned (nothing launched) once
 * a plan's support reaches beyond that; create the ensemble again then. */
int cmbx_ensemble_launch(cmbx_ensemble* ens, void* stream);
/* Release an ensemble (waits for the device first). NULL is accepted. */
int cmbx_ensemble_destroy(cmbx_ensemble* ens);

/* ---- stage-by-stage entry points (tests and profiling) ---- */

/* The 768 binary32 entries of the single-precision Box-Muller tables, computed on the host
 * (no device needed): ln(1 + j/128), or ln((1 + j/128)/2) for j >= 54, then 1/(1 + j/128)
 * for j = 0..127, then sin and cos of (k + 1/2) 2 pi/256 for k = 0..255, each the binary64
 * value rounded once. The noise of Sec. II D 1 in FP32 plans reads them. out: host buffer
 * of cap >= 768 floats. Returns 768, or CMBX_EINVAL. */
int cmbx_noise_tables(float* out, int cap);

/* Write the unpacked weighted half grid of realisation `seed`: device complex array
 * [N][N][N/2+1] of the plan's precision (re, im interleaved). */
int cmbx_debug_noise(cmbx_plan* plan, uint64_t seed, void* halfgrid);
/* Run noise + inverse FFT for one realisation into `field`: device real [N][N][N]. */
int cmbx_debug_field(cmbx_plan* plan, uint64_t seed, void* field);
/* Run the first `npasses` (1..3) kernels of the field computation for realisation `seed`
 * into `buf` (device, N^3 reals of the plan's precision). After pass 1 (x) and pass 2 (y)
 * buf holds complex [N][N][N/2]: the half grid transformed along x (and y), with column
 * iz = 0 carrying Z(iz=0) + i Z(iz=N/2), except where the spectrum's support makes the
 * result zero and the next pass does not read it (those entries are left as they were);
 * after pass 3 it is the real field. */
int cmbx_debug_passes(cmbx_plan* plan, uint64_t seed, int npasses, void* buf);
/* Size in bytes of a map footprint for box size N (CMBX_EINVAL outside [8, 1024]). */
int64_t cmbx_footprint_bytes(int N);
/* The map footprint of (r, dirs) as cmbx_simulate_patch makes it on a pruning plan, into
 * fp (device, cmbx_footprint_bytes(N) bytes, 4-byte aligned; the bytes past the list's
 * count are left as they were). Layout: bytes [0, N) flag the x-planes ix some pixel's
 * stencil reads; then, per ix, ceil(N/8) bytes flag the 8-row blocks iy/8 of its lines
 * (ix, iy) that some stencil reads; then ceil(N/32) bytes flag the 32-node blocks iz/32
 * of z that some stencil reads (1 read, 0 not); then, at the next multiple of 4 bytes,
 * uint32 [lines, z count, plane count, 0], then N^2 slots of which the first z count hold
 * the blocks of `lines` consecutive (ix, iy) lines (lines = the plan's z tile) with a
 * flagged line, then N slots of which the first plane count hold the flagged planes; each
 * entry once, in no particular order. Errors: CMBX_EINVAL (r out of range, n_pix, NULL or misaligned). */
int cmbx_debug_footprint(cmbx_plan* plan, double r, const double* dirs, int64_t n_pix, void* fp);
/* Interpolate a caller-given device field [N][N][N] (plan precision, 16-byte aligned) at
 * the pixels. CMBX_EINVAL for a misaligned field. */
int cmbx_debug_gather(cmbx_plan* plan, const void* field, double r, const double* dirs,
                      int64_t n_pix, void* out);

/*
 * Time each kernel of the hot path for realisation `seed` of the plan (its first batch
 * slot): every kernel is launched once untimed and then `reps` times in a row on the
 * plan's stream between two HIP events (the first timed launch is queued while the
 * untimed one runs), and ms[i] receives the average duration in milliseconds of kernel
 * i: ms[0] pass x (noise + x transform), ms[1] pass y, ms[2] pass z (complex-to-real),
 * ms[3] gather into out[0 .. n_pix). The passes run as in cmbx_simulate_patch: if the
 * plan prunes, the map footprint is made first, and with CMBX_OPT_FIXED_DIRS the pixel
 * order (neither timed). The y and z passes work in
 * place, so their repeated launches touch the same memory as one launch but leave no
 * realisation behind: simulate again before using the workspace or out. Synchronises the
 * plan's stream. Errors: as cmbx_simulate_patch, CMBX_EINVAL for reps < 1 or ms == NULL.
 */
int cmbx_time_passes(cmbx_plan* plan, uint64_t seed, double r, const double* dirs, int64_t n_pix,
                     void* out, int reps, double* ms);

/*
 * Autotune the plan's workgroup shapes and FFT stage plans by coordinate descent (two
 * sweeps over the x, y and z pass): each compiled choice of one pass -- every tile
 * (cmbx_tile_choices) with stage plan 0, and the default tile with stage plan 1 where
 * compiled -- the other two held at their best so far, is timed with HIP events over
 * `reps` runs of the whole x -> y -> z chain on the plan's stream (one pass's write pattern
 * changes the cost of the next, so a kernel timed alone can mislead); the fastest chain's
 * shapes and plans become the plan's options (cmbx_plan_get reads them back). best[0..2] receives (tile_x, tile_y, lines_z) and ms[0..2] the average
 * milliseconds of each pass alone at those shapes (either may be NULL). Needs a spectrum
 * (CMBX_ESTATE otherwise); overwrites the first workspace slot; synchronises the plan's
 * stream.
 */
int cmbx_plan_autotune(cmbx_plan* plan, int reps, int* best, double* ms);
/* As cmbx_plan_autotune, but on a pruning plan the chains are timed as maps of these pixels
 * (r, dirs, n_pix as in cmbx_simulate_patch) are made: from their footprint, whose z list
 * is rebuilt for each z tile tried (not timed). Which shapes win depends on how much of
 * the field the map reads. Leaves the footprint in the plan. */
int cmbx_plan_autotune_patch(cmbx_plan* plan, int reps, double r, const double* dirs, int64_t n_pix,
                             int* best, double* ms);
/* Compiled tile choices for (dtype, N): which = 0 for the x/y column tiles, 1 for the z
 * lines. Writes up to 4 values to out and returns their count (0 if none). */
int cmbx_tile_choices(int dtype, int N, int which, int* out);

/*
 * Enqueue one stage of the hot path for realisation `seed` on `stream` (a hipStream_t;
 * NULL = the null stream), for callers that schedule the stages themselves (e.g. on
 * streams restricted to different compute units). stage 0: noise + x pass into buf;
 * 1: y pass on buf; 2: z pass on buf; 3: gather from buf (r, dirs, n_pix, out as in
 * cmbx_simulate_patch; ignored by stages 0-2). buf: device, N^3 reals of the plan's
 * precision, 16-byte aligned. Tile shapes are the plan's; stages 0-2 make the whole field
 * (no map footprint). Errors: CMBX_ESTATE (no
 * spectrum), CMBX_EINVAL, CMBX_EHIP.
 */
int cmbx_enqueue_stage(cmbx_plan* plan, int stage, uint64_t seed, void* buf, double r, const double* dirs,
                       int64_t n_pix, void* out, void* stream);

/* ---- flat boxes: the 3-D method on N x N x M and the 2-D (hybrid) method ----
 * Sec. II C sizes the box as N x N points across and M along the line of sight z, all
 * spaced dp, so P_box = P_inf (2 pi / dp)^3 / (M N^2) (eq. finalpbox) at
 * |k| = (2 pi / dp) sqrt((fx^2 + fy^2) / N^2 + fz^2 / M^2). A slab plan makes nz layers of
 * such a box, real [nz][N][N] (y fastest), node (ix, iy, j) at (ix dp, iy dp, j dp),
 * periodic in x and y:
 *   CMBX_SLAB_FLAT   -- the 3-D Fourier method (Sec. II D 1) on the whole N x N x M box,
 *                       nz = M, periodic in z. Modes of the half grid in y (iy = 0 .. N/2,
 *                       all ix, iz) from Philox counter (iz >> 1, iy, ix, 2), words
 *                       (x0, x1) / (x2, x3) for even / odd iz, the canonical Box-Muller
 *                       of the plan precision; generic modes sqrt(P_box / 2) (g_re + i g_im);
 *                       on the planes iy = 0, N/2 the mode and (-ix, -iz) are conjugate
 *                       (the smaller ix M + iz drawn), the self-conjugate ones real,
 *                       sqrt(P_box) g_re. Field: the unnormalised + sign inverse DFT.
 *   CMBX_SLAB_HYBRID -- the 2-D Fourier method (Sec. II D 2): only the layers j = 0 .. h-1
 *                       (nz = h <= 32), made in hybrid space (k_x, k_y, z): per column the
 *                       h values are S g, S the symmetric square root P D^{1/2} P^T of the
 *                       column covariance Gamma_jk = xi(|j - k| dp), xi the transform
 *                       along z of P_box over the M values of f_z (eq. gammasvd; same
 *                       statistics as P D^{1/2}, unique), formed once per spectrum on the
 *                       host in FP64 (Jacobi eigendecomposition, negative eigenvalues of
 *                       rounding set to 0) and rounded to the plan precision; g: h normal
 *                       pairs from Philox counter (j >> 1, iy, ix, 1), divided by sqrt 2
 *                       for generic columns, the real part only for the four
 *                       self-conjugate ones; rows iy = 0, N/2 Hermitian in x. Then the
 *                       inverse 2-D DFT of every layer.
 * Pixels: p = (r n + o) (1 / dp) per axis in FP64; x, y wrap modulo N; z wraps modulo M on
 * the flat box, and on the hybrid layers a pixel whose stencil leaves [0, h) is NaN
 * (place the layers about the cap with cmbx_slab_observer). Default observer: the middle
 * of the layers, (N dp / 2, N dp / 2, (nz - 1) dp / 2).
 * Sizes: N as for cmbx_plan_box (2^a 3^b, 8 .. 1024); flat: M even, 2^a 3^b, 8 .. 512;
 * hybrid: 2 <= M (even), 1 <= h <= min(M, 32); nz N a multiple of a compiled z tile. */
#define CMBX_SLAB_FLAT   1
#define CMBX_SLAB_HYBRID 2
typedef struct cmbx_slab cmbx_slab;

/* Create a slab plan (method, N, M, h (ignored for CMBX_SLAB_FLAT: h = M), dp > 0, dtype,
 * batch >= 1). It owns batch x nz x N^2 reals of workspace, the twiddles and, once a
 * spectrum is set, the per-column tables. Errors: CMBX_EINVAL, CMBX_EUNSUPPORTED (sizes not
 * compiled), CMBX_ENOMEM, CMBX_EHIP. */
int cmbx_slab_create(int method, int N, int M, int h, double dp, int dtype, int batch, cmbx_slab** out);
int cmbx_slab_destroy(cmbx_slab* slab);
/* CMBX_OPT_INTERP and CMBX_OPT_STREAM as for plans, and CMBX_SLAB_OPT_DIRECT: how a map's
 * values are taken from the layers. After the transform along x, each (layer, x) line holds
 * its half spectrum along y, and the value at row y is that line's inverse DFT at y; with
 * CMBX_SLAB_DIRECT_ALWAYS every stencil row is summed directly from it (N/2 terms, the
 * plan's twiddles) instead of running the complex-to-real pass over every line and then
 * the gather; CMBX_SLAB_DIRECT_NEVER always runs the pass; CMBX_SLAB_DIRECT_AUTO (default)
 * sums directly while n_pix K^2 N/2 <= 2 nz N^2 (K = 4 tricubic, 2 trilinear). The maps
 * agree to rounding. CMBX_EINVAL for other keys or values. */
#define CMBX_SLAB_OPT_DIRECT    12
#define CMBX_SLAB_DIRECT_AUTO   0
#define CMBX_SLAB_DIRECT_NEVER  1
#define CMBX_SLAB_DIRECT_ALWAYS 2
int cmbx_slab_set(cmbx_slab* slab, int key, int64_t value);
/* Observer position o in box coordinates (the length unit of dp and r); CMBX_EINVAL if not
 * finite. Sec. II D 2 centres the h layers on the cap: o_z = (h - 1) dp / 2 - r (1 + z_min) / 2. */
int cmbx_slab_observer(cmbx_slab* slab, double x, double y, double z);
/* The observer that centres the slab's nz layers on a cap (Sec. II D 2, Fig. 2b): the cap
 * about +z at radius r > 0 with edge z_min in [-1, 1]; xyz = (N dp / 2, N dp / 2,
 * (nz - 1) dp / 2 - r (1 + z_min) / 2), written to xyz (host); nothing changes. CMBX_EINVAL
 * for a bad r, z_min or NULL xyz. */
int cmbx_slab_cap_observer(const cmbx_slab* slab, double r, double z_min, double* xyz);
/* Spectrum as for cmbx_spectrum_table: host FP64 k (increasing), P_inf (>= 0), n >= 2,
 * linear between nodes, zero outside. Builds the per-column tables (FP64, rounded once);
 * synchronises the slab's stream. */
int cmbx_slab_spectrum(cmbx_slab* slab, const double* k, const double* P_inf, int64_t n);
/* Maps of the batch (realisation b uses seed + b) at the pixels: dirs device FP64
 * [n_pix][3], out device [batch][n_pix] of the plan precision; asynchronous on the
 * slab's stream; the layers of the last realisation stay in the workspace (transformed
 * along x only, complex [nz][N][N/2], when the map was summed directly). Errors:
 * CMBX_ESTATE (no spectrum), CMBX_EINVAL (r <= 0 or not finite, n_pix, NULL), CMBX_EHIP. */
int cmbx_slab_simulate(cmbx_slab* slab, uint64_t seed, double r, const double* dirs, int64_t n_pix, void* out);
/* Tests: the layers of realisation `seed`, real [nz][N][N] (device, plan precision); the
 * column stage alone, unpacked: flat, the modes [N][N/2+1][M]; hybrid, the correlated
 * columns [h][N][N/2+1] (device complex of the plan precision). */
int cmbx_slab_debug_layers(cmbx_slab* slab, uint64_t seed, void* layers);
int cmbx_slab_debug_columns(cmbx_slab* slab, uint64_t seed, void* cols);
/* Hybrid slabs with a spectrum: the FP64 factor S (h x h, row-major, host) of the columns
 * with fx^2 + fy^2 = s, as the library formed it before rounding. CMBX_EINVAL if s is not a
 * sum of two squares of 0 .. N/2 or the slab is flat. */
int cmbx_slab_factor(const cmbx_slab* slab, int64_t s, double* S);
/* Layers, rows and pixels of a slab: any pointer may be NULL. */
int cmbx_slab_info(const cmbx_slab* slab, int* N, int* M, int* nz, double* dp, void** layers);
/* The box sizing rule of Sec. II C for a beam b (radians) and cap theta_max (radians) on a
 * sphere of radius R: dp = 0.85 R b / 5 (0.85 of the programme's constraint spacing); N and
 * M are size_factor times the next power of two of twice the cap's width 2 R sin(theta_max)
 * and twice its height R (1 - cos theta_max) in points (host only). CMBX_EINVAL for
 * non-positive or non-finite arguments. */
int cmbx_box_size(double b, double theta_max, double size_factor, double R, int* N, int* M, double* dp);

/* ---- sky pixels ----
 * HEALPix pixel centres of the cap centred on the pole (Sec. II D 1: for a cap about the
 * pole the pixels to sample are the leading pixels of a HEALPix map in RING order;
 * pixelization of Gorski et al., ApJ 622 (2005) 759). Resolution nside (1 .. 2^20): 12
 * nside^2 pixels on rings 1 .. 4 nside - 1 from the pole. The cap holds every ring whose
 * height z is >= z_min (z_min = cos theta_max); each ring's z is one correctly rounded
 * FP64 quotient of integers, (3n^2 - i^2) / (3n^2) for polar rings and (4n - 2i) / (3n)
 * for the others (south rings: the negated mirror), so the cut is reproducible.
 * Sets *n_pix (host pointer, required) to the cap's pixel count. If dirs is not NULL
 * (device memory, caller-owned, room for `capacity` pixels of 3 FP64 each), enqueues on
 * `stream` (a hipStream_t; NULL = the null stream) the unit directions in RING order,
 * (sin t cos phi, sin t sin phi, z) with sin t = sqrt((1 - z)(1 + z)): the `dirs` that
 * cmbx_simulate_patch and the ensembles take. With dirs NULL the call touches no device.
 * Errors: CMBX_EINVAL (n_pix NULL, nside out of range, z_min NaN, capacity < *n_pix: the
 * count is still set), CMBX_EHIP. */
int cmbx_healpix_cap(int64_t nside, double z_min, double* dirs, int64_t capacity, int64_t* n_pix, void* stream);

/* ---- covariance test of the maps ----
 * Pixel covariance of a sky map with angular power spectrum C_l (Sec. III B tests the
 * maps against it; eq. harmonics): gamma[i][j] = sum_{l=0}^{lmax} (2l + 1) C_l
 * P_l(n_i . n_j) / (4 pi), with n_i . n_j clamped to [-1, 1], for i, j < n_pix, FP64,
 * row-major. dirs ([n_pix][3] unit directions), cl (lmax + 1 values) and gamma
 * (n_pix^2 values) are device memory, caller-owned; enqueued on `stream` (a hipStream_t,
 * NULL = the null stream). P_l comes from the three-term recurrence in FP64. Whitening and
 * the KS test on the result are left to the caller. Errors: CMBX_EINVAL (NULL pointer,
 * n_pix outside [1, 1048560], lmax outside [0, 65536]), CMBX_EHIP. */
int cmbx_pixel_covariance(const double* dirs, int64_t n_pix, const double* cl, int lmax, double* gamma,
                          void* stream);

/* Whitening of maps for the covariance test (Sec. III B): with Gamma + s^2 I = L L^T, the
 * vector x = L^-1 m of a map m (plus white noise of variance s^2) should hold independent
 * unit normals, which the caller tests (Kolmogorov-Smirnov). FP64, device memory,
 * row-major, enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *
 * cmbx_cholesky: A (n x n, leading dimension lda >= n) is overwritten in its lower triangle
 * by the factor L of A + shift I (blocked, 64-wide panels; the trailing updates on the
 * FP64 matrix cores); the strict upper triangle is left as it was. info (device int64,
 * may be NULL) receives 0, or the 1-based column of the first pivot that is not positive
 * (the matrix plus shift is not positive definite; the factor then holds NaN).
 * cmbx_whiten: every row of B (nrhs x n, leading dimension ldb >= n; one map per row) is
 * replaced by L^-1 row, for L from cmbx_cholesky (leading dimension ldl).
 * cmbx_gemm_nt_sub: C (m x n) -= A (m x k) B (n x k)^T, k <= 64 (the building block of both;
 * lower != 0 writes only the entries on or below the diagonal).
 * Errors: CMBX_EINVAL (NULL, sizes < 1, leading dimensions too short, k out of range),
 * CMBX_EHIP. */
int cmbx_cholesky(double* A, int64_t n, int64_t lda, double shift, int64_t* info, void* stream);
int cmbx_whiten(const double* L, int64_t n, int64_t ldl, double* B, int64_t nrhs, int64_t ldb, void* stream);
int cmbx_gemm_nt_sub(int64_t m, int64_t n, int k, const double* A, int64_t lda, const double* B, int64_t ldb,
                     double* C, int64_t ldc, int lower, void* stream);

/* ---- spectrum surrogate network (Sec. II B inversion, learned) ----
 * Building blocks of a small MLP that maps a C_l vector to a P_inf table. All pointers are
 * device memory, row-major, caller-owned; work is enqueued on `stream` (NULL = null
 * stream). Errors: CMBX_EINVAL for non-positive sizes, NULL pointers or leading
 * dimensions shorter than a row; CMBX_EHIP for launch failures. */

/* C = op(A) op(B) (+ bias), Y = GELU(C) (act = 1) or C (act = 0; Y may be NULL).
 * op(A) is M x K: A is FP32, stored M x K (lda >= K) or, with transA, K x M (lda >= M).
 * op(B) is K x N: B is BF16 (b_bf16 = 1, raw 16-bit words) or FP32, stored K x N
 * (ldb >= N) or, with transB, N x K (ldb >= K). Both operands are rounded to BF16 (nearest
 * even) and multiplied on the matrix cores with FP32 accumulation. GELU is the exact
 * x Phi(x). C is M x N FP32 (ldc >= N); bias has N values or is NULL. */
int cmbx_mlp_gemm(int M, int N, int K, const float* A, int lda, int transA, const void* B, int ldb,
                  int transB, int b_bf16, float* C, int ldc, const float* bias, int act, float* Y,
                  int ldy, void* stream);
/* dZ = dY * GELU'(Z), elementwise over n values. */
int cmbx_mlp_gelu_backward(const float* Z, const float* dY, float* dZ, int64_t n, void* stream);
/* out[c] = sum_r X[r][c] for a rows x cols matrix (the bias gradient). */
int cmbx_mlp_colsum(const float* X, int rows, int cols, float* out, void* stream);
/* Mean squared error over n values: dY = 2 (Y - T) / n and *loss = mean (Y - T)^2 (device
 * scalar); `partial` is device scratch of at least cmbx_mlp_mse_partials(n) floats. */
int cmbx_mlp_mse(const float* Y, const float* T, int64_t n, float* dY, float* partial, float* loss,
                 void* stream);
int64_t cmbx_mlp_mse_partials(int64_t n);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * training loops, harnesses that forbid hipMalloc): cmbx_mlp_mse with its partial sums in a
 * static device array of the library (256 KiB per device, held until the process ends)
 * instead of a caller's workspace. Allocates nothing. Same arguments and results as
 * cmbx_mlp_mse without `partial`; n at most CMBX_MSE_NOALLOC_MAX (CMBX_EINVAL beyond).
 * Every call on one device shares that device's array, so calls that overlap on a device
 * (other streams, other threads) race; calls ordered on one stream do not. */
#define CMBX_MSE_NOALLOC_MAX (65536ll * 256)
int cmbx_mlp_mse_noalloc(const float* Y, const float* T, int64_t n, float* dY, float* loss, void* stream);
/* One Adam step (Kingma & Ba) on n FP32 master weights w with moments m, v and gradient g
 * at step `step` >= 1; writes the BF16 copy w_bf16 (raw 16-bit words) if not NULL. */
int cmbx_mlp_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float beta1,
                  float beta2, float eps, int step, uint16_t* w_bf16, void* stream);
/* y = BF16(x), round to nearest even, n values. */
int cmbx_bf16_round(const float* x, uint16_t* y, int64_t n, void* stream);

/* Message of the calling thread's last failed call ("" if none). Valid until its next call. */
const char* cmbx_last_error(void);
/* Library version string. */
const char* cmbx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CMBX_H */
