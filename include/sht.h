/*
 * sht.h -- C ABI of an MI355X (gfx950) spherical-harmonic transform library.
 *
 * The transform is the one the ESCAPE D3.3 spectral-transform dwarf is built
 * on (report section 4.4.1, defining equation repeated in 4.4.2): a field on a
 * Gaussian grid is a Fourier series in longitude whose coefficient for zonal
 * wavenumber m is a Legendre sum over total wavenumber n of the spectral
 * coefficients a_n^m times the normalised associated Legendre functions
 * Pbar_n^m(mu), mu = cos(colatitude).  Section 4.2 describes the same
 * transform as two stages per direction -- per-latitude FFTs in longitude
 * and one Legendre matrix product per m -- with all latitudes, wavenumbers
 * and fields exposed to the GPU at once (4.2.2-4.2.3), arrays allocated
 * once outside the time loop (4.2.3) and no device synchronisation between
 * calls (4.2.5).  This library keeps that structure.
 *
 * Directions:
 *   inverse  (synthesis)  spectral -> grid
 *   direct   (analysis)   grid -> spectral
 *
 * Conventions (the report leaves these unstated; this library fixes them):
 *   - integral over mu in [-1, 1] of Pbar_n^m squared is 1; no
 *     Condon-Shortley phase;
 *   - real fields: only m >= 0 is stored; Im a_n^0 is ignored on input and
 *     written as exactly 0 on output;
 *   - triangular truncation: 0 <= m <= n <= N;
 *   - Gaussian latitudes are the roots of P_nlat, ordered north to south;
 *     point k of a ring of n points is at longitude 2 pi k / n;
 *   - per-ring Fourier truncation mmax_j = min(N, floor((nlon_j - 1) / 2));
 *   - analysis is Gaussian quadrature: a_n^m = sum_j w_j chat_{j,m}
 *     Pbar_n^m(mu_j) with chat_{j,m} = (1/nlon_j) sum_k g_{j,k} e^{-i m lam_k}.
 *
 * Grids:
 *   SHT_GRID_FULL        nlat = N + 1 rings of 2N + 2 points (N must be odd,
 *                        so that every ring has a mirror ring)
 *   SHT_GRID_OCTAHEDRAL  O(N + 1): nlat = 2(N + 1) rings; ring i counted
 *                        from either pole has 20 + 4i points
 *
 * Precisions:
 *   SHT_FP64    data, tables, FFT and Legendre products in float64
 *               (FP64 MFMA)
 *   SHT_FP32    data, tables, FFT in float32; Legendre products on FP32 MFMA
 *   SHT_BF16X3  data and FFT in float32; Legendre products with both
 *               operands split x = hi + lo (bfloat16, round to nearest even)
 *               and three BF16 MFMA products hi*hi + hi*lo + lo*hi
 *               accumulated in float32
 *   Latitudes, weights and Pbar are always computed in float64 on the GPU
 *   at plan time and rounded once to the table type.
 *
 * Layouts (all arrays are device memory owned by the caller unless stated):
 *   spectral  [F][nspec] complex, real and imaginary parts interleaved,
 *             nspec = (N+1)(N+2)/2, m-major triangular:
 *             index(m, n) = m (2N + 3 - m) / 2 + (n - m).
 *   grid      [F][npts] real, rings north to south, ring j at ring_offset[j].
 *   element type is double for SHT_FP64, float otherwise.
 *
 *   Fourier workspace, synthesis form (written by sht_legendre_inverse,
 *   read by sht_fourier_synthesis): for ring j (0..nlat-1), wavenumber
 *   m (0..mmax_j) and field f, the complex coefficient c_{j,m} of field f
 *   is at complex index (four_row[j] + m) * fpad + f, with
 *   four_row[j] = sum_{i<j} (mmax_i + 1) and fpad = F rounded up to 16.
 *
 *   Fourier workspace, analysis form (written by sht_fourier_analysis,
 *   read by sht_legendre_direct): for north ring j (0..nlat/2-1), m and
 *   slot p the complex value is at ((four_row[j] + m) * 2 + p) * fpad + f:
 *   slot 0 holds (w_j/nlon_j) chat(ring j), slot 1 (w_j/nlon_j)
 *   chat(mirror ring).  sht_legendre_direct forms the symmetric and
 *   antisymmetric parts S = slot 0 + slot 1 and A = slot 0 - slot 1.
 *
 * Ownership and concurrency: a plan owns its device tables and metadata and
 * is immutable after creation.  sht_inverse / sht_direct and the stage calls
 * never allocate and never synchronise the host; they enqueue on the given
 * HIP stream (NULL = the default stream) and return.  Concurrent calls on
 * one plan are safe if each has its own workspace and outputs.
 *
 * Errors: every call returns SHT_OK (0) or a negative code; nothing throws
 * across the ABI.  After SHT_EHIP, sht_last_hip_error() returns the HIP
 * error code of the failing call (per thread).
 */
#ifndef SHT_H
#define SHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum sht_grid { SHT_GRID_FULL = 0, SHT_GRID_OCTAHEDRAL = 1 };
enum sht_prec { SHT_FP64 = 0, SHT_FP32 = 1, SHT_BF16X3 = 2 };

enum sht_status {
  SHT_OK = 0,
  SHT_EINVAL = -1,       /* bad argument (null pointer, out-of-range value) */
  SHT_EUNSUPPORTED = -2, /* (truncation, grid, precision) not supported     */
  SHT_ENOMEM = -3,       /* device allocation failed at plan creation       */
  SHT_EHIP = -4,         /* a HIP call failed; see sht_last_hip_error()     */
  SHT_ESCRATCH = -5      /* sht_transform_static: the plan's workspace is
                            larger than SHT_STATIC_SCRATCH_BYTES            */
};

/* Transform directions (sht_transform_static). */
enum sht_direction { SHT_DIR_INVERSE = 0, SHT_DIR_DIRECT = 1 };

/* Size of the per-device scratch array behind sht_transform_static. */
#define SHT_STATIC_SCRATCH_BYTES (64u << 20)

typedef struct sht_plan_s* sht_plan_t;

typedef struct sht_info {
  int32_t truncation; /* N */
  int32_t grid;       /* enum sht_grid */
  int32_t nfields;    /* F */
  int32_t precision;  /* enum sht_prec */
  int32_t nlat;       /* number of rings */
  int32_t fpad;       /* F rounded up to 16: field stride of the workspace */
  int64_t npts;       /* grid points per field */
  int64_t nspec;      /* spectral coefficients per field */
  int64_t nfour;      /* sum over rings of (mmax_j + 1) */
  int64_t workspace_bytes;
  int64_t table_bytes;   /* resident Pbar tables */
  int64_t plan_bytes;    /* device bytes of the plan, shared tables included */
  int32_t elem_bytes;    /* 8 for SHT_FP64, 4 otherwise */
  int32_t tile;          /* Legendre column-tile variant in use (enum sht_tile) */
  int64_t own_bytes;     /* device bytes of the plan without the shared tables */
  int32_t vector;        /* 1 for plans of sht_plan_create_vector, else 0 */
  int32_t degree;        /* highest degree of the Pbar tables: N, or N + 1 for vector plans */
  int32_t table_free;    /* 1 for plans of sht_plan_create_table_free, else 0 */
  int32_t reserved;
  int64_t chunk_table_bytes; /* table-free plans: bytes of one chunk's tables (in the workspace) */
} sht_info;

/* Pointwise spectral operators (sht_spectral_op), on the unit sphere. */
enum sht_op {
  SHT_OP_DLAMBDA = 0,      /* d/dlambda:  a_n^m -> i m a_n^m                 */
  SHT_OP_LAPLACIAN = 1,    /* Laplacian:  a_n^m -> -n (n + 1) a_n^m           */
  SHT_OP_INV_LAPLACIAN = 2 /* its inverse: a_n^m -> -a_n^m / (n (n + 1)), 0 at n = 0 */
};

/* Column-tile variants of the Legendre products: the 2F real columns of a
 * product are cut into tiles of 128, 64 or 32 columns.  FP32 and FP64 plans
 * start with 32 columns when 2F <= 32, else 64 (FP64: 64 or 32 only).
 * BF16X3 plans start with C128 (MFMA 32x32x16: synthesis tiles of 128 rings
 * x 128 columns, analysis tiles of 128 k x 128 columns); C64 selects tiles of
 * 128 rings x 64 columns and 64 k x 128 columns (MFMA 16x16x32). */
enum sht_tile { SHT_TILE_C128 = 0, SHT_TILE_C64 = 1, SHT_TILE_C32 = 2 };

typedef struct sht_batch_s* sht_batch_t;

/* Batch flags. */
enum sht_batch_flags {
  SHT_BATCH_PERSISTENT = 1, /* each Legendre launch uses only as many work groups as stay
                               resident, each looping over the concatenated work list (FFT
                               launches always give each (ring, field) its own work group) */
  SHT_BATCH_GRAPH = 2       /* capture the stage launches in a HIP graph on first use, replay after */
};

/* Create a plan: geometry, Gaussian latitudes and weights (Newton iteration
 * on P_nlat in float64), Pbar_n^m tables (float64 recurrence, rounded once
 * to the table type), FFT twiddle and chirp tables, and the Legendre work
 * lists.  Every table is computed by kernels on `hip_stream`; the call
 * synchronises that stream once before returning.  `truncation` >= 1 (odd
 * for SHT_GRID_FULL), `nfields` >= 1.  On success *out receives the plan. */
int sht_plan_create(sht_plan_t* out, int truncation, int grid, int nfields,
                    int precision, void* hip_stream);

/* A plan that keeps no Pbar tables resident, for truncations whose tables
 * would not fit the device (they grow as N^3: 3.6 GB in FP32 at TCo1279,
 * ~0.5 TB at T8191): the wavenumbers are cut into chunks whose tables fit
 * `chunk_bytes` (0: 256 MiB; a wavenumber whose tables alone are larger is
 * a chunk by itself), and each transform makes a chunk's tables in its workspace
 * (float64 recurrence, the same kernel and values as the resident tables
 * of sht_plan_create) right before that chunk's Legendre product.  Results
 * are bitwise those of a plan from sht_plan_create with the same arguments
 * (same tables, same product kernels and summation order); each transform
 * pays for making the tables.  Arguments and errors as sht_plan_create.
 * Serves sht_inverse, sht_direct, the stage calls (which then need the
 * whole workspace: sht_workspace_size covers the Fourier buffer and one
 * chunk's tables), sht_stepper_*; not batches, sht_plan_legendre_table or
 * sht_transform_static beyond its scratch. */
int sht_plan_create_table_free(sht_plan_t* out, int truncation, int grid, int nfields, int precision,
                               size_t chunk_bytes, void* hip_stream);

/* A plan for `nfields` fields that shares every device table of `base`
 * (same truncation, grid and precision): only its descriptor and work lists
 * are new, so it is cheap to make and holds little memory.  The tables stay
 * allocated until the last plan sharing them is destroyed; `base` may be
 * destroyed first.  Synchronises `hip_stream`.  For callers that serve many
 * field counts from resident tables. */
int sht_plan_create_like(sht_plan_t* out, sht_plan_t base, int nfields, void* hip_stream);

/* Release a plan and its device memory (synchronises the device first). */
int sht_plan_destroy(sht_plan_t plan);

/* Release a plan in stream order, without synchronising: its device memory
 * (and the shared tables, if this was the last plan holding them) is freed
 * on `hip_stream` after the work enqueued there before the call.  The caller
 * guarantees that no work on other streams still uses the plan (for example
 * by waiting for an event of its last transform first).  For serving loops
 * that must not stall every stream to drop one plan. */
int sht_plan_destroy_async(sht_plan_t plan, void* hip_stream);

/* Sizes of a plan (host struct, no device work). */
int sht_plan_info(sht_plan_t plan, sht_info* out);

/* Copy the plan's geometry to host arrays of nlat entries each (any may be
 * NULL): latitudes mu, Gaussian weights w, ring lengths nlon, per-ring
 * Fourier truncation mmax, and four_row (nlat + 1 entries: row offsets of
 * the Fourier workspace).  ring_offset receives nlat + 1 grid offsets.
 * Synchronous. */
int sht_plan_geometry(sht_plan_t plan, double* mu, double* w, int32_t* nlon,
                      int32_t* mmax, int64_t* ring_offset, int64_t* four_row);

/* Copy the resident Pbar table of wavenumber m to host as float64,
 * [rows][N - m + 1] with rows = the north rings that carry m (mmax_j >= m),
 * pole to equator; *first_ring receives the index of the first such ring.
 * For SHT_BF16X3 the value is hi + lo.  `out` must hold rows * (N-m+1)
 * doubles where rows = nlat/2 - *first_ring; pass out = NULL to query
 * first_ring only.  Synchronous.  For tests of the plan kernels. */
int sht_plan_legendre_table(sht_plan_t plan, int m, double* out, int32_t* first_ring);

/* Bytes of workspace sht_inverse / sht_direct need (the Fourier buffer). */
size_t sht_workspace_size(sht_plan_t plan);

/* Synthesis of all F fields: spectral -> grid.  `spec` [F][nspec] complex,
 * `grid` [F][npts] real, `workspace` >= sht_workspace_size bytes, all device
 * pointers aligned to 16 bytes.  Enqueues sht_legendre_inverse then
 * sht_fourier_synthesis on the stream.  Asynchronous. */
int sht_inverse(sht_plan_t plan, const void* spec, void* grid, void* workspace,
                void* hip_stream);

/* Analysis of all F fields: grid -> spectral.  Enqueues
 * sht_fourier_analysis then sht_legendre_direct.  Asynchronous. */
int sht_direct(sht_plan_t plan, const void* grid, void* spec, void* workspace,
               void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform as sht_inverse (direction SHT_DIR_INVERSE, `in` = spec, `out` =
 * grid) or sht_direct (SHT_DIR_DIRECT, `in` = grid, `out` = spec), with the
 * workspace taken from a fixed array of SHT_STATIC_SCRATCH_BYTES that the
 * library holds in each GPU's memory (reserved when the library is loaded,
 * kept until the process ends) instead of from the caller.  Results are
 * bitwise those of sht_inverse / sht_direct.  Calls no allocating routine;
 * the first call on a device looks the array's device address up once.
 * SHT_ESCRATCH if sht_workspace_size(plan) exceeds the array (64 MiB holds,
 * for example, T399 full grid with up to 16 fields in FP64, or TCo399 with
 * up to 16 fields in FP32).  Every call on one GPU shares that GPU's array:
 * calls whose executions overlap on one GPU (other streams, other threads)
 * race and give undefined results; order them.  Asynchronous, like
 * sht_inverse. */
int sht_transform_static(sht_plan_t plan, int direction, const void* in, void* out, void* hip_stream);

/* ---- Derivatives and vector (wind) transforms ----
 *
 * The report works in spectral space because derivatives become pointwise
 * multiplications there (section 4.4.1).  On the unit sphere (multiply
 * winds by 1/a, vorticity and divergence by 1/a for radius a), with
 * mu = sin(latitude), U = u cos(lat), V = v cos(lat), stream function psi
 * and velocity potential chi (vorticity zeta = Lap psi, divergence
 * D = Lap chi):
 *   U = dchi/dlambda - (1 - mu^2) dpsi/dmu,
 *   V = dpsi/dlambda + (1 - mu^2) dchi/dmu.
 * The mu derivative is taken in spectral space with the derivative identity
 *   (1 - mu^2) dPbar_n^m/dmu = (n+1) e_n Pbar_{n-1}^m - n e_{n+1} Pbar_{n+1}^m,
 *   e_n = sqrt((n^2 - m^2) / (4 n^2 - 1)),
 * so U and V are syntheses of degree up to N + 1 with the Pbar tables
 * alone (extended by one degree).  The analysis is the Gaussian quadrature
 * below with a second table, H_n^m = (1 - mu^2) dPbar_n^m/dmu of degree
 * <= N, computed in float64 from the same identity at plan time (forming
 * the H sums from Pbar projections of neighbouring degrees instead would
 * cancel, and multiply the rounding of the products by up to ~N).
 * zeta_0^0 and D_0^0 do not enter the winds and are returned as 0; Im of
 * every m = 0 coefficient is ignored on input and 0 on output.
 *
 * Layouts: vortdiv [2][F][nspec] complex (the F vorticity fields, then the
 * F divergence fields), uv [2][F][npts] real (the F U fields, then the F V
 * fields), nspec and npts of truncation N. */

/* A plan for F vector fields (2F grid components): Pbar tables to degree
 * N + 1 and H tables to degree N (each the size of a scalar plan's table),
 * the analysis weight w_j / (1 - mu_j^2) per ring, work lists for 2F
 * components.  Arguments and errors as sht_plan_create.  Such a plan serves
 * sht_vector_inverse, sht_vector_direct, sht_gradient and sht_spectral_op;
 * the scalar calls (sht_inverse, stages, batches) reject it with
 * SHT_EINVAL.  sht_plan_create_like makes a vector plan from a vector
 * base.  Its sht_workspace_size covers the Fourier buffer of 2F components
 * and two arrays of 2F wind coefficients of degree N + 1. */
int sht_plan_create_vector(sht_plan_t* out, int truncation, int grid, int nfields,
                           int precision, void* hip_stream);

/* Winds from vorticity and divergence: vortdiv [2][F][nspec] -> uv
 * [2][F][npts].  Asynchronous on `hip_stream`; no allocation. */
int sht_vector_inverse(sht_plan_t plan, const void* vortdiv, void* uv, void* workspace,
                       void* hip_stream);

/* Vorticity and divergence from winds: uv [2][F][npts] -> vortdiv
 * [2][F][nspec], by Gaussian quadrature:
 *   zeta_n^m = sum_j w_j/(1-mu_j^2) [i m V_{j,m} Pbar_n^m(mu_j) + U_{j,m} H_n^m(mu_j)],
 *   D_n^m    = sum_j w_j/(1-mu_j^2) [i m U_{j,m} Pbar_n^m(mu_j) - V_{j,m} H_n^m(mu_j)],
 * H = (1 - mu^2) dPbar/dmu, U_{j,m}, V_{j,m} the ring DFT coefficients
 * (1/nlon_j) sum_k (.) e^{-i m lambda_k}.  Asynchronous; no allocation. */
int sht_vector_direct(sht_plan_t plan, const void* uv, void* vortdiv, void* workspace,
                      void* hip_stream);

/* cos(lat) times the gradient of F scalar fields: spec [F][nspec] -> uv
 * [2][F][npts] with U = df/dlambda, V = (1 - mu^2) df/dmu (the wind of
 * velocity potential f).  Asynchronous; no allocation. */
int sht_gradient(sht_plan_t plan, const void* spec, void* uv, void* workspace, void* hip_stream);

/* `op` (enum sht_op) on `count` spectral fields [count][nspec] of the plan's
 * truncation and data type; in == out is allowed.  Asynchronous. */
int sht_spectral_op(sht_plan_t plan, int op, int count, const void* in, void* out, void* hip_stream);

/* ---- Time stepping ----
 *
 * The loop a spectral model runs (report sections 4.2.2-4.2.3: synthesis,
 * grid-point computations and analysis every time step, with every array
 * allocated once outside the loop), here for the reaction-diffusion
 * equation du/dt = nu Lap u + r u (1 - u) on the unit sphere, by
 * semi-implicit Euler steps of length dt: the logistic term explicit on the
 * grid, the diffusion implicit in spectral space,
 *   g = synthesis(a);  g <- g + dt r g (1 - g);  b = analysis(g);
 *   a_n^m <- b_n^m / (1 + dt nu n (n + 1)).
 * The grid-point step is applied as the synthesis stores the grid, and the
 * diffusion as the analysis stores the coefficients (each value rounded
 * once after the transform's own rounding): a step is the four stages.
 * A stepper binds a scalar plan to the state `spec` ([F][nspec], updated in
 * place every step), a grid and a workspace (scratch).  With SHT_STEP_GRAPH
 * `graph_steps` consecutive steps are captured once into a HIP graph on
 * `hip_stream` (which must not be NULL) and replayed: one launch per
 * graph_steps steps instead of one per kernel.  The buffers must outlive
 * the stepper. */
typedef struct sht_stepper_s* sht_stepper_t;
enum sht_step_flags { SHT_STEP_GRAPH = 1 };

/* dt >= 0, nu >= 0, all finite; 1 <= graph_steps <= 4096 (ignored
 * without SHT_STEP_GRAPH).  Captures (no kernel runs) when SHT_STEP_GRAPH
 * is set. */
int sht_stepper_create(sht_stepper_t* out, sht_plan_t plan, double dt, double rate, double nu, void* spec,
                       void* grid, void* workspace, int flags, int graph_steps, void* hip_stream);

/* Enqueue `nsteps` time steps on `hip_stream` (asynchronous): nsteps /
 * graph_steps graph replays, then the remaining steps kernel by kernel. */
int sht_stepper_run(sht_stepper_t stepper, int nsteps, void* hip_stream);

/* Release a stepper (synchronises the device first if it holds a graph). */
int sht_stepper_destroy(sht_stepper_t stepper);

/* Stage 1 of synthesis: per m, S_m = Pbar_even a_even and A_m = Pbar_odd
 * a_odd over the north rings carrying m, then c(ring j) = S + A and
 * c(mirror ring) = S - A, written in the synthesis form of the Fourier
 * workspace (report 4.2.4: the Legendre transform as matrix products). */
int sht_legendre_inverse(sht_plan_t plan, const void* spec, void* fourier,
                         void* hip_stream);

/* Stage 2 of synthesis: per ring, the real inverse DFT of c_{j,0..mmax_j}
 * (zero above mmax_j) onto the ring's nlon_j points (report 4.2.5). */
int sht_fourier_synthesis(sht_plan_t plan, const void* fourier, void* grid,
                          void* hip_stream);

/* Stage 1 of analysis: per ring, the real DFT and the (w_j / nlon_j)
 * scaling, written in the analysis form of the Fourier workspace. */
int sht_fourier_analysis(sht_plan_t plan, const void* grid, void* fourier,
                         void* hip_stream);

/* Stage 2 of analysis: per m, a_n^m = Pbar^T S (n - m even) or Pbar^T A
 * (n - m odd) summed over the north rings carrying m, with S and A formed
 * from the two slots of the analysis form. */
int sht_legendre_direct(sht_plan_t plan, const void* fourier, void* spec,
                        void* hip_stream);

/* Switch a plan's Legendre products to another column-tile variant (results
 * are unchanged: every output keeps its summation order).  Synchronises
 * `hip_stream`.  SHT_EINVAL if the variant is not available for the plan's
 * precision. */
int sht_plan_set_tile(sht_plan_t plan, int tile, void* hip_stream);

/* Batches: many independent transforms of uneven truncation and field count
 * run in shared launches -- one launch per stage (per tile variant present
 * for the Legendre products, per work-group kind present for the FFTs) over
 * the concatenation of every plan's work list, ordered by cost, largest
 * first.  This is the report's batching of
 * the Legendre products across the second spherical dimension (section
 * 4.2.4) taken one step further: across transforms, with each product at
 * its own size instead of zero-padding to a common one, and its wish for an
 * FFT batched over differing sizes (section 4.2.5) for all rings of all
 * transforms at once.
 *
 * All plans must have the same precision and outlive the batch.  The batch
 * owns only its work lists and descriptor tables. */
int sht_batch_create(sht_batch_t* out, const sht_plan_t* plans, int n, int flags, void* hip_stream);

/* Workspace bytes for the whole batch (the plans' workspaces, 256-byte
 * aligned, back to back). */
size_t sht_batch_workspace_size(sht_batch_t batch);

/* Bind the device buffers of every transform: spec[i] and grid[i] in plan
 * i's layouts, one workspace of sht_batch_workspace_size bytes.  The small
 * device descriptor table is rewritten by a kernel enqueued on `hip_stream`,
 * so the new binding takes effect in stream order: runs enqueued on that
 * stream before the call keep the buffers they were bound to, runs after it
 * use the new ones (no host synchronisation).  Runs on other streams must
 * be ordered by the caller.  A captured graph reads the table, so it stays
 * valid across rebinding. */
int sht_batch_bind(sht_batch_t batch, void* const* spec, void* const* grid, void* workspace,
                   void* hip_stream);

/* Synthesis / analysis of every transform of the batch on `hip_stream`
 * (asynchronous).  SHT_EINVAL before the first sht_batch_bind. */
int sht_batch_inverse(sht_batch_t batch, void* hip_stream);
int sht_batch_direct(sht_batch_t batch, void* hip_stream);

/* Autotuner: for each distinct (truncation, grid, fields) of the batch, time
 * the two Legendre products with every tile variant available and keep the
 * fastest; rebuilds the work lists (and drops a captured graph).  Reads the
 * bound spectral inputs, uses the bound workspace as scratch and a
 * temporary array for analysis output: bound inputs and outputs are left as
 * they were.  Allocates temporaries; synchronises `hip_stream`. */
int sht_batch_tune(sht_batch_t batch, void* hip_stream);

/* The tile variant chosen for each plan of the batch (n entries). */
int sht_batch_tiles(sht_batch_t batch, int32_t* out);

/* Set each plan's tile variant (n entries of enum sht_tile, e.g. choices
 * sht_batch_tune made in an earlier run and kept by the caller) and rebuild
 * the work lists; drops a captured graph.  SHT_EINVAL if a variant is not
 * available for the batch's precision.  Synchronises `hip_stream`. */
int sht_batch_set_tiles(sht_batch_t batch, const int32_t* tiles, void* hip_stream);

int sht_batch_destroy(sht_batch_t batch);

/* Human-readable text of a status code. */
const char* sht_strerror(int status);

/* HIP error code of the last SHT_EHIP on this thread (0 if none). */
int sht_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SHT_H */
