/*
 * fftpl.h -- C ABI of the MI355X (gfx950) hot path of FFTPL, the FFT-based
 * electrostatic global placer of J. Lu et al., "FFTPL: An Analytic Placement
 * Algorithm Using Fast Fourier Transform for Density Equalization".
 *
 * One evaluation of the placement objective f = W~ + lambda*N (Eq. (7)) and
 * its gradient: cells are rasterised into an n x n bin density map (Eq. (2)),
 * the Neumann Poisson equation (Eq. (8)) is solved spectrally (Eqs. (9)-(12)),
 * the field is gathered back to the cells (Section III-C), and the weighted-
 * average wirelength gradient (Eq. (3)) is added.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array pointer is a DEVICE pointer owned by the caller.  The library
 *   never frees, retains or copies caller memory beyond the call.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *   compute call only enqueues work on `stream` and returns; no call
 *   synchronises the host, and no compute call allocates device memory
 *   (workspace lives in the plan).  fftpl_eval may also run part of its work
 *   on the plan's own stream, forked from `stream` and joined back into it
 *   with events, so its results are ordered on `stream` like any other.
 * - Every call returns an int status (enum fftpl_status) and never throws.
 *   Argument errors are detected on the host before anything is enqueued and
 *   return FFTPL_E_INVAL.  A failed kernel launch returns FFTPL_E_DEVICE;
 *   because launches are asynchronous, a fault of earlier work may also be
 *   reported as FFTPL_E_DEVICE by a later call.
 * - Units: positions, sizes, bin sizes and gamma are physical; maps are in
 *   bin-area units (a full bin has density 1).  Maps are float32 row-major
 *   [iy][ix] with ix (the x direction) fastest, n*n entries.
 * - Cell rectangles: each cell's edges in bin units are computed in float32,
 *   one rounding per operation and no contraction:
 *       c = (x - (float)xl) * (float)(1/bin_w);  half = 0.5f * (w * (float)(1/bin_w));
 *       lo = c - half;  hi = c + half
 *   Bins are half-open [j, j+1); a cell touches bins floor(lo) .. ceil(hi)-1,
 *   clipped to [0, n-1]; its overlap with bin j is min(hi, j+1) - max(lo, j)
 *   with the edges clipped to [0, n].  Cells outside the region contribute
 *   only their in-region part.
 * - A plan is not thread-safe; use one plan per stream.
 * - Setting the environment variable FFTPL_VALIDATE=1 adds O(pins) content
 *   checks (CSR monotone, pin cells in range, positive sizes) that copy the
 *   arrays to the host and synchronise; they are off by default.
 */
#ifndef FFTPL_H
#define FFTPL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFTPL_VERSION 20100 /* major*10000 + minor*100 + patch */

enum fftpl_status {
  FFTPL_OK = 0,
  FFTPL_E_INVAL = -1,       /* bad argument (NULL, size, mode, n)           */
  FFTPL_E_NOMEM = -2,       /* device allocation failed (plan creation)     */
  FFTPL_E_DEVICE = -3,      /* a HIP runtime call or kernel launch failed   */
  FFTPL_E_UNSUPPORTED = -4, /* valid but not supported (e.g. n for a mode)  */
  FFTPL_E_STATE = -5        /* plan used with a grid of another size        */
};

/* How the DCT/DST stages of the spectral solve are computed. */
enum fftpl_dct_mode {
  FFTPL_DCT_FFT = 0,         /* hand-written radix-4 FFTs in LDS, float32     */
  FFTPL_DCT_GEMM_F32 = 1,    /* cosine/sine-matrix GEMMs on MFMA, float32     */
  FFTPL_DCT_GEMM_BF16X3 = 2  /* the same GEMMs with each float32 operand split
                                into bf16 hi + lo, three MFMA products
                                (hi*hi + hi*lo + lo*hi), float32 accumulate   */
};

/* Which density gradient is produced. */
enum fftpl_grad_mode {
  FFTPL_GRAD_FIELD = 0, /* Section III-C: dN/dx_i ~ -q_i E_i, with the cell's
                           field the overlap-weighted sum of E over its bins */
  FFTPL_GRAD_EXACT = 1  /* exact derivative of N = sum_b rho_b psi_b (Eq. (6))
                           with respect to the cell centre (includes the
                           factor 2 of the quadratic form)                   */
};

/* Wirelength model of the objective. */
enum fftpl_wl_model {
  FFTPL_WL_WA = 0, /* weighted average, Eq. (3): the paper's model          */
  FFTPL_WL_LSE = 1 /* log-sum-exp, the smooth model Section II names beside
                      Eq. (3): per net and axis
                      gamma ln sum e^(X/gamma) + gamma ln sum e^(-X/gamma)  */
};

/* The bin grid over the placement region R (Section II): n x n bins of
 * bin_w x bin_h starting at (xl, yl).  target_density is rho_t, the scale of
 * fixed-node charge (Section III-B). */
typedef struct fftpl_grid {
  int32_t n;
  int32_t reserved; /* must be 0 */
  double xl, yl;
  double bin_w, bin_h;
  double target_density;
} fftpl_grid;

/* Opaque: twiddle/trigonometric tables and map workspace for one n, one
 * dct_mode and up to max_batch designs evaluated together (fftpl_eval_batch).
 * About 36*n*n bytes of device memory per batch slot at n = 1024. */
typedef struct fftpl_plan fftpl_plan;

/* A static netlist and fixed charge; references caller-owned device arrays,
 * the library copies nothing.  w, h: movable cell sizes [num_cells].
 * base: fixed charge map [n*n] (see fftpl_fixed_map) or NULL for none.
 * cap: movable capacity map [n*n] for the overflow ratio, or NULL to use
 * max(0, rho_t - min(rho_t, base)).  Nets: CSR net_ptr [num_nets+1]
 * (net_ptr[0] = 0, nondecreasing, net_ptr[num_nets] = num_pins), pin_cell
 * [num_pins] in [0, num_cells), pin offsets from the cell centre
 * pin_dx, pin_dy [num_pins].
 *
 * Optional, for the atomic-free evaluation paths (n <= 1024): a device
 * workspace `work` of work_bytes >= fftpl_problem_work_bytes(...) bytes, owned
 * by the caller and used by one evaluation at a time, and one pin index
 * (work and xindex 256-byte aligned, as device allocations are; otherwise
 * fftpl_eval returns FFTPL_E_INVAL):
 *   - the exchange index (fastest): xindex / xindex_bytes from
 *     fftpl_xindex_build for this netlist and max_degree, and xindex_key, the
 *     key that build returned;
 *   - or the cell-major slots: cell_ptr [num_cells+1] and pin_slot
 *     [num_pins] from fftpl_netlist_index.
 * With neither work nor an index fftpl_eval uses float atomics for the density
 * scatter and the wirelength gradient (fftpl_problem_path reports which path
 * a problem takes).  A workspace or an index that is given but cannot be
 * used is an error, never a silent change of path: FFTPL_E_UNSUPPORTED for
 * n > 1024, FFTPL_E_INVAL for a missing or too small workspace or index,
 * FFTPL_E_STATE when xindex_key does not match the sizes, max_degree,
 * net_ptr, pin_cell and xindex of the problem (an index built for another
 * netlist).  All paths give the same results up to float32 rounding order.
 * An index must be rebuilt when net_ptr or pin_cell change; pin offsets and
 * positions may change freely.
 *
 * wl_model selects the wirelength term W~ (enum fftpl_wl_model; 0 is the
 * paper's weighted average).  screening is eps >= 0 of the screened solve
 * (see fftpl_helmholtz_solve; 0 is the paper's Poisson equation). */
typedef struct fftpl_problem {
  fftpl_grid grid;
  int32_t num_cells;
  int32_t num_nets;
  int32_t num_pins;
  int32_t wl_model; /* enum fftpl_wl_model */
  const float* w;
  const float* h;
  const float* base;
  const float* cap;
  const int32_t* net_ptr;
  const int32_t* pin_cell;
  const float* pin_dx;
  const float* pin_dy;
  const int32_t* cell_ptr;
  const int32_t* pin_slot;
  void* work;
  uint64_t work_bytes;
  const void* xindex;
  uint64_t xindex_bytes;
  int32_t max_degree; /* the value xindex was built for */
  float screening;    /* eps >= 0, bin^-2 units; 0 = Poisson */
  uint64_t xindex_key; /* returned by fftpl_xindex_build for xindex */
} fftpl_problem;

/* Which implementation of the density scatter and the wirelength gradient an
 * evaluation of a problem takes (fftpl_problem_path). */
enum fftpl_path {
  FFTPL_PATH_EXCHANGE = 0, /* banded LDS scatter, bucketed pin exchange:
                              no float atomics, bit-repeatable              */
  FFTPL_PATH_SLOTS = 1,    /* banded LDS scatter, cell-major pin slots      */
  FFTPL_PATH_ATOMIC = 2    /* float atomics for both (no workspace, no index) */
};

/* Library version (FFTPL_VERSION of the build). */
int fftpl_version(void);

/* Static, NUL-terminated description of a status code. */
const char* fftpl_status_string(int status);

/* Create a plan for grid side n, a dct_mode and batches of up to max_batch
 * designs (1 <= max_batch <= FFTPL_MAX_BATCH; fftpl_eval_batch evaluates that
 * many designs in one launch per stage).  FFTPL_DCT_FFT needs n a power of two
 * with 8 <= n <= 1024 (the paper's grids are powers of two up to 1024, Section
 * IV-A); the GEMM modes need n a multiple of 64 with 64 <= n <= 4096.  Tables
 * are uploaded on `stream`.  On success *out owns device memory until
 * fftpl_plan_destroy.  Errors: FFTPL_E_INVAL (NULL out, bad mode or
 * max_batch), FFTPL_E_UNSUPPORTED (n), FFTPL_E_NOMEM, FFTPL_E_DEVICE. */
#define FFTPL_MAX_BATCH 8
int fftpl_plan_create(fftpl_plan** out, int32_t n, int32_t dct_mode, int32_t max_batch,
                      void* stream);

/* Destroy a plan (synchronises the device first).  NULL is accepted. */
int fftpl_plan_destroy(fftpl_plan* plan);

/* Side n, dct_mode and max_batch of a plan (any output may be NULL). */
int fftpl_plan_info(const fftpl_plan* plan, int32_t* n, int32_t* dct_mode,
                    int32_t* max_batch);

/* Device pointers of the maps the last fftpl_eval on this plan produced, for
 * inspection: rho [n*n], psi [n*n] (written in FFTPL_GRAD_EXACT mode), exy
 * [2*n*n]: in FFTPL_GRAD_FIELD mode (Ex, Ey) interleaved per bin; in
 * FFTPL_GRAD_EXACT mode the differences of psi to the next bin centre,
 * (psi[iy][ix+1] - psi[iy][ix], psi[iy+1][ix] - psi[iy][ix]), computed in the
 * spectral domain (Section III-C: the exact gradient sums them; taking them
 * as differences of rounded psi values would lose their leading digits).
 * Owned by the plan.  Any pointer argument may be NULL.  After
 * fftpl_eval_batch the maps of the batch's request i follow at offsets
 * i*n*n (rho, psi) and i*2*n*n (exy) floats from these pointers, for the
 * requests evaluated together in the call's last group (see
 * fftpl_eval_batch). */
int fftpl_plan_maps(const fftpl_plan* plan, const float** rho, const float** psi,
                    const float** exy);

/* Per-kernel timing for profiling.  With enable = 1 every later
 * fftpl_poisson_solve / fftpl_eval on this plan records a HIP event on its
 * stream after each kernel (and one before the first).  Creates the events on
 * first use. */
int fftpl_plan_timing(fftpl_plan* plan, int32_t enable);

/* Durations of the kernels of the last timed call on this plan, in launch
 * order: ms[i] and names[i] (static strings) for i < *count <= max.  Waits for
 * the last event.  *count = 0 when timing is off. */
int fftpl_plan_kernel_times(fftpl_plan* plan, int32_t max, float* ms, const char** names,
                            int32_t* count);

/* Fixed charge (Section III-B: fixed and dark node areas scaled by rho_t):
 *   base[b] = rho_t * f_b,  cap[b] = rho_t * max(0, 1 - min(1, f_b)),
 * f_b = sum over fixed rectangles of their overlap with bin b.  Rectangles
 * are given by centre (fx, fy) and size (fw, fh) [num_fixed].  base is
 * overwritten; cap may be NULL.  num_fixed may be 0 (maps become 0 and rho_t). */
int fftpl_fixed_map(const fftpl_grid* grid, int32_t num_fixed, const float* fx,
                    const float* fy, const float* fw, const float* fh, float* base,
                    float* cap, void* stream);

/* Dark nodes of an irregular placement region (Section III-B: each
 * non-placeable rectangle inside the bounding box R is a dark node, charged
 * like a fixed node at the target density).  Host-only: given R = [xl, xh] x
 * [yl, yh] and the placeable part as the union of num_rects rectangles
 * (HOST array rects [4*num_rects] of corners x0, y0, x1, y1 with x0 <= x1 and
 * y0 <= y1; clipped to R, overlaps allowed), writes R minus that union as
 * disjoint rectangles to the HOST array out [4*max_out] (same corner layout)
 * and their count to *num_out.  The pieces are horizontal slabs between
 * consecutive distinct y edges, merged upwards while the x intervals stay the
 * same.  Rasterise them with fftpl_fixed_map (centre and size per
 * rectangle) beside any fixed macros; a macro overlapping a dark node is
 * counted twice there.  More than max_out pieces: FFTPL_E_INVAL with
 * *num_out = the number needed (call again with a larger out).  Non-finite
 * values, an inverted rectangle or an empty R: FFTPL_E_INVAL. */
int fftpl_dark_nodes(double xl, double yl, double xh, double yh, int32_t num_rects,
                     const double* rects, int32_t max_out, double* out, int32_t* num_out);

/* Density map (Eq. (2), Section III-B): rho = base + sum over movable cells of
 * their overlap area with each bin.  base may be NULL (treated as 0).  rho is
 * overwritten.  For n <= 1024 it runs the evaluation's banded scatter
 * (counting sort by band, fixed-point LDS sums: the same bits on every run)
 * with its band lists in a temporary allocation made and released on
 * `stream` (hipMallocAsync / hipFreeAsync; FFTPL_E_NOMEM if it fails); the
 * caller that keeps a workspace uses fftpl_problem_density, the caller that
 * cannot allocate fftpl_density_map_noalloc.  For n > 1024 it accumulates
 * with float atomics: the rounding order (not the value beyond float32
 * rounding) then varies between runs. */
int fftpl_density_map(const fftpl_grid* grid, int32_t num_cells, const float* x,
                      const float* y, const float* w, const float* h,
                      const float* base, float* rho, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * density map of fftpl_density_map with the same arguments, computed like
 * fftpl_problem_density (banded counting sort, fixed-point LDS sums: rho is
 * the same on every run) with the band lists in a static device array of
 * FFTPL_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call allocates nothing.  At most
 * FFTPL_NOALLOC_MAX_CELLS cells and n <= 1024 (FFTPL_E_UNSUPPORTED
 * otherwise).  Every call on one GPU uses that GPU's one array: calls that
 * overlap on a GPU (other streams, other threads) race and must be ordered
 * by the caller. */
#define FFTPL_NOALLOC_SCRATCH_BYTES (64 << 20)
#define FFTPL_NOALLOC_MAX_CELLS 921600
int fftpl_density_map_noalloc(const fftpl_grid* grid, int32_t num_cells, const float* x,
                              const float* y, const float* w, const float* h,
                              const float* base, float* rho, void* stream);

/* The density map of a problem's cells at positions x, y [num_cells], the
 * same quantity as fftpl_density_map with grid, w, h and base from prob,
 * computed without float atomics in prob->work (banded counting sort of the
 * cells, fixed-point sums in LDS): rho [n*n] is the same on every run.  Needs
 * prob->work (FFTPL_E_INVAL otherwise) and n <= 1024
 * (FFTPL_E_UNSUPPORTED).  The netlist fields of prob are not read. */
int fftpl_problem_density(const fftpl_problem* prob, const float* x, const float* y,
                          float* rho, void* stream);

/* Path an evaluation of prob takes (enum fftpl_path) into *path, or the
 * status fftpl_eval would return for the problem's workspace and index
 * fields.  Host-only; reads no device memory. */
int fftpl_problem_path(const fftpl_problem* prob, int32_t* path);

/* Spectral Neumann Poisson solve (Eqs. (8)-(12)) on the plan's grid:
 *   a_uv = (c_u c_v / n^2) sum rho cos(w_u (ix+1/2)) cos(w_v (iy+1/2)),
 *   c_0 = 1, c_{k>0} = 2, w_u = pi u / n, a_00 := 0 (DC removed, Section III-A),
 *   psi = sum a/(w_u^2+w_v^2) cos cos, Ex = sum a w_u/(..) sin(w_u x) cos(w_v y),
 *   Ey = sum a w_v/(..) cos(w_u x) sin(w_v y), at bin centres, bin units.
 * rho is read; psi, ex, ey [n*n] are written (ex and ey may both be NULL);
 * energy, if not NULL, is a device double set to N = sum_b rho_b psi_b
 * (Eq. (6)).  grid->n must equal the plan's n (else FFTPL_E_STATE). */
int fftpl_poisson_solve(fftpl_plan* plan, const fftpl_grid* grid, const float* rho,
                        float* psi, float* ex, float* ey, double* energy,
                        void* stream);

/* The screened (Helmholtz) form of the solve, Eq. (4) as Section II cites
 * it, taken with the sign convention of Eq. (8):
 *   -laplace(psi) + eps psi = rho - mean(rho)   (Neumann boundary),
 * i.e. every mode of fftpl_poisson_solve is divided by w_u^2 + w_v^2 + eps
 * instead of w_u^2 + w_v^2 (eps in bin^-2 units, like w_u^2; the DC is still
 * removed).  eps = 0 is fftpl_poisson_solve.  eps must be finite and >= 0
 * (else FFTPL_E_INVAL); the other arguments are those of
 * fftpl_poisson_solve. */
int fftpl_helmholtz_solve(fftpl_plan* plan, const fftpl_grid* grid, float eps,
                          const float* rho, float* psi, float* ex, float* ey,
                          double* energy, void* stream);

/* Density gradient per movable cell (Section III-C), times `scale` (lambda):
 *   FIELD: gx_i = -scale/bin_w * sum_b ov(i,b) Ex_b  (gy with Ey, bin_h); reads ex, ey.
 *   EXACT: gx_i = 2*scale/bin_w * sum_iy oy(i,iy) [psi(iy, floor(hi)) [0<hi<n]
 *                                              - psi(iy, floor(lo)) [0<lo<n]]
 *          (gy symmetric); reads psi.
 * accumulate = 0 overwrites gx, gy; 1 adds to them. */
int fftpl_field_gather(const fftpl_grid* grid, int32_t num_cells, const float* x,
                       const float* y, const float* w, const float* h,
                       const float* ex, const float* ey, const float* psi,
                       int32_t grad_mode, float scale, int32_t accumulate,
                       float* gx, float* gy, void* stream);

/* Weighted-average wirelength (Eq. (3)) and HPWL (Eq. (1)) over the pin-net
 * CSR, pins at cell centre + offset.  Adds (accumulate = 1) or writes
 * (accumulate = 0) dW~/dx, dW~/dy summed over each cell's pins into gx, gy
 * [num_cells].  wa and hpwl, if not NULL, are device doubles set to the
 * totals over all nets and both axes.  gamma > 0, physical units.  Each pin's
 * gradient is added to its cell in 64-bit fixed point (units of 2^-32; a
 * non-finite pin gradient makes its cell NaN) and the totals are per-block
 * partials summed in a fixed order, so the results are the same on every
 * run; the accumulators live in a temporary allocation made and released on
 * `stream` (hipMallocAsync / hipFreeAsync; FFTPL_E_NOMEM if it fails).  The
 * per-cell adds are global atomics (one per pin and axis); the problem form
 * fftpl_problem_wl_grad moves the pins through its exchange index instead. */
int fftpl_wa_grad(int32_t num_nets, const int32_t* net_ptr, int32_t num_pins,
                  const int32_t* pin_cell, const float* pin_dx, const float* pin_dy,
                  int32_t num_cells, const float* x, const float* y, float gamma,
                  int32_t accumulate, float* gx, float* gy, double* wa,
                  double* hpwl, void* stream);

/* The log-sum-exp wirelength (FFTPL_WL_LSE) with the arguments, outputs and
 * errors of fftpl_wa_grad: per net and axis, with M, L the largest and
 * smallest pin coordinate, S+ = sum exp((X - M)/gamma), S- = sum exp((L -
 * X)/gamma): value (M - L) + gamma (ln S+ + ln S-), gradient
 * exp((X_p - M)/gamma)/S+ - exp((L - X_p)/gamma)/S-.  wa receives the LSE
 * total. */
int fftpl_lse_grad(int32_t num_nets, const int32_t* net_ptr, int32_t num_pins,
                   const int32_t* pin_cell, const float* pin_dx, const float* pin_dy,
                   int32_t num_cells, const float* x, const float* y, float gamma,
                   int32_t accumulate, float* gx, float* gy, double* wa, double* hpwl,
                   void* stream);

/* The wirelength term of a problem (prob->wl_model: Eq. (3) or log-sum-exp)
 * at positions x, y [num_cells]: adds (accumulate = 1) or writes
 * (accumulate = 0) each cell's summed pin gradient into gx, gy [num_cells];
 * wl and hpwl, if not NULL, are device doubles set to the totals.  The same
 * quantities as fftpl_wa_grad / fftpl_lse_grad, through the bucketed pin
 * exchange of prob->xindex (its key in prob->xindex_key) in prob->work,
 * without float atomics: the result is the same on every run.  Errors as for
 * an evaluation of prob (FFTPL_E_INVAL without work or xindex,
 * FFTPL_E_STATE for an index of another netlist); gamma > 0. */
int fftpl_problem_wl_grad(const fftpl_problem* prob, const float* x, const float* y,
                          float gamma, int32_t accumulate, float* gx, float* gy, double* wl,
                          double* hpwl, void* stream);

/* Bytes of the optional fftpl_problem workspace for grid side n, num_cells
 * cells, num_nets nets and num_pins pins (the interleaved positions, per-pin
 * gradients, band lists of the density scatter, their counters, and per-block
 * partial sums of the wirelength).  Host-only. */
int fftpl_problem_work_bytes(int32_t n, int32_t num_cells, int32_t num_nets,
                             int32_t num_pins, uint64_t* bytes);

/* Cell-major index of the pins of a netlist (Section II: the netlist as a
 * hypergraph; this is the transpose of its pin-net incidence), built once per
 * netlist on `stream`:
 *   cell_ptr [num_cells+1]: cell_ptr[c] = number of pins on cells < c,
 *   pin_slot [num_pins]:    a permutation of 0..num_pins-1 with
 *                           cell_ptr[pin_cell[p]] <= pin_slot[p] < cell_ptr[pin_cell[p]+1].
 * The order of one cell's slots is arbitrary (integer atomics) but fixed once
 * built.  work: device int32 scratch of num_cells + (num_cells+1023)/1024 + 1
 * entries.  pin_cell values must lie in [0, num_cells). */
int fftpl_netlist_index(int32_t num_cells, int32_t num_pins, const int32_t* pin_cell,
                        int32_t* cell_ptr, int32_t* pin_slot, int32_t* work, void* stream);

/* Exchange index of a netlist (Section II: the netlist as a hypergraph; the
 * index is a blocked form of the transpose of its pin-net incidence), for the
 * fastest fftpl_eval path.  Cells are cut into blocks of consecutive cells
 * (a multiple of 256 cells, at most 9216, about one block per compute unit)
 * and nets into blocks of whole nets (at most 9728 pins per block); the
 * index lists the pins by (cell block, net block) and, per net block, by cell
 * block, so that positions and gradients move between cells and nets in runs
 * through on-chip memory.
 *
 * fftpl_xindex_bytes: device bytes of the index and of the build's scratch
 * for num_cells cells, num_nets nets, num_pins pins and nets of degree at most
 * max_degree.  Host-only.  FFTPL_E_UNSUPPORTED when max_degree > 8705.
 *
 * fftpl_xindex_build: builds the index into `index` (index_bytes, caller
 * owned, 256-byte aligned; valid until net_ptr or pin_cell change) using
 * `work` (work_bytes, 256-byte aligned, free again on return), on `stream`,
 * and waits for it (the call synchronises the stream).  *key (if key is not
 * NULL) receives a host-side fingerprint of the sizes, max_degree and the
 * net_ptr, pin_cell and index pointers; a problem using the index carries it
 * in xindex_key, so that an index built for another netlist is refused on the
 * host without reading device memory.  FFTPL_E_INVAL when a net has more than
 * max_degree pins, when net_ptr is not a CSR over num_pins pins or when a
 * pin_cell lies outside [0, num_cells); the index is then unusable. */
int fftpl_xindex_bytes(int32_t num_cells, int32_t num_nets, int32_t num_pins,
                       int32_t max_degree, uint64_t* index_bytes, uint64_t* work_bytes);
int fftpl_xindex_build(int32_t num_cells, int32_t num_nets, int32_t num_pins,
                       const int32_t* net_ptr, const int32_t* pin_cell, int32_t max_degree,
                       void* index, uint64_t index_bytes, void* work, uint64_t work_bytes,
                       uint64_t* key, void* stream);

/* One full evaluation (Algorithm 1, the density / FFT solve / gradient steps):
 *   rho = base + cells; Poisson solve (screened when prob->screening > 0);
 *   g = dW~/dv + lambda * g_N (grad_mode; W~ per prob->wl_model);
 *   out4 (device double[4]) = [N, W~, HPWL, tau] with tau the overflow ratio
 *   sum_b max(0, rho_b - base_b - cap_b) / sum_b (rho_b - base_b).
 * gx, gy [num_cells] are overwritten.  prob->grid.n must equal the plan's n.
 * With gx = gy = NULL only out4 is computed (the loss W~ + lambda N and the
 * other scalars, without the gather); this needs a workspace and an index in
 * prob (FFTPL_E_INVAL otherwise).  A workspace or index that prob gives but
 * that cannot be used is an error (see fftpl_problem), not a silent change
 * of path.  With a workspace and an index the
 * wirelength branch (pin positions, net blocks) runs on the plan's own stream
 * concurrently with the density branch (scatter, solve, per-cell density
 * gradient) on `stream`, and is joined back before the per-cell sums; the
 * density map, the
 * cell sums and the scalars do not depend on the order of any atomic adds,
 * so repeated evaluations give identical results. */
int fftpl_eval(fftpl_plan* plan, const fftpl_problem* prob, const float* x,
               const float* y, float lambda, float gamma, int32_t grad_mode,
               float* gx, float* gy, double* out4, void* stream);

/* fftpl_eval with lambda and gamma read on the device, when the kernels run,
 * from params[0] and params[1] (a device float[2]) instead of host arguments,
 * so that a loop whose lambda and gamma are set on the device
 * (fftpl_nesterov_schedule) can be enqueued, or captured in a graph, with no
 * host read per iteration.  The results are those of fftpl_eval(..., params[0],
 * params[1], ...): the same kernels and arithmetic (1/gamma formed in float as
 * on the host).  Exchange path only (a problem with a workspace and an
 * index; FFTPL_E_UNSUPPORTED otherwise); gx and gy must not be NULL.  params
 * is read on the device and not checked: it must hold a finite lambda and a
 * finite gamma > 0 when the evaluation runs (otherwise the results are not
 * finite). */
int fftpl_eval_params(fftpl_plan* plan, const fftpl_problem* prob, const float* x,
                      const float* y, const float* params, int32_t grad_mode, float* gx,
                      float* gy, double* out4, void* stream);

/* Serving extension: count evaluations of designs that share the plan's grid
 * side, with the results of
 *   fftpl_eval(plan, probs[i], xs[i], ys[i], lambdas[i], gammas[i], grad_mode,
 *              gxs ? gxs[i] : NULL, gys ? gys[i] : NULL, out4s + 4*i, stream)
 * for every i.  probs, xs, ys, lambdas, gammas, gxs and gys are HOST arrays of
 * count entries (gxs and gys both NULL: the scalars only, for every request);
 * the pointers they hold and out4s (double [4*count]) are device memory.
 * Requests are taken in order in groups of up to the plan's max_batch that
 * take the exchange path, have workspaces that do not overlap and share the
 * wirelength model and net-block size class; each group runs every stage
 * (scatter, the three FFT passes, field gather, pin exchange, per-cell sums)
 * as one launch over all of its designs (GEMM plans run the solve of each
 * design in turn inside the group).  Requests that cannot join a group run
 * alone.  Every request is checked on the host before anything is enqueued:
 * on an argument error nothing runs and the status of the first failing
 * request is returned.  count = 0 is a no-op. */
int fftpl_eval_batch(fftpl_plan* plan, int32_t count, const fftpl_problem* const* probs,
                     const float* const* xs, const float* const* ys, const float* lambdas,
                     const float* gammas, int32_t grad_mode, float* const* gxs,
                     float* const* gys, double* out4s, void* stream);

/* Placement iteration (Algorithm 1: after each evaluation the positions move
 * along the gradient).  The global placement here uses Nesterov's method with
 * a look-ahead point u at which the gradient g is taken; the step length is
 * chosen on the host from these statistics (all device, double):
 *   out4 = [sum (u - u_prev)^2, sum (g - g_prev)^2, max |g|, sum |g|]
 * over both axes of num_cells cells.  upx, upy, gpx, gpy may all be NULL (the
 * first iteration: out4[0] = out4[1] = 0).  work: device double scratch of at
 * least 1024 entries (work_doubles).  Per-block partials summed in a fixed
 * order: repeatable. */
int fftpl_step_stats(int32_t num_cells, const float* ux, const float* uy, const float* upx,
                     const float* upy, const float* gx, const float* gy, const float* gpx,
                     const float* gpy, double* out4, double* work, uint64_t work_doubles,
                     void* stream);

/* The Nesterov update of every cell centre (device arrays [num_cells]):
 *   x_new = clamp(u - step g),  u_new = clamp(x_new + beta (x_new - x)),
 *   then u_prev = u, g_prev = g, x = x_new, u = u_new,
 * with clamp keeping the cell (sizes w, h) inside the region of `region`
 * ([xl, xl + n bin_w] x [yl, yl + n bin_h]; a cell wider than the region
 * sits at its centre).  step >= 0, 0 <= beta < 1. */
int fftpl_nesterov_update(const fftpl_grid* region, int32_t num_cells, const float* w,
                          const float* h, float* x, float* y, float* ux, float* uy, float* upx,
                          float* upy, float* gpx, float* gpy, const float* gx, const float* gy,
                          float step, float beta, void* stream);

/* fftpl_nesterov_update with step and beta read on the device from
 * step_beta[0] and step_beta[1] (device doubles, rounded to float like the
 * host call's arguments; e.g. state + 12 of fftpl_nesterov_schedule).  Not
 * checked on the host: step >= 0 and 0 <= beta < 1 are the schedule's to
 * keep. */
int fftpl_nesterov_update_dev(const fftpl_grid* region, int32_t num_cells, const float* w,
                              const float* h, float* x, float* y, float* ux, float* uy,
                              float* upx, float* upy, float* gpx, float* gpy, const float* gx,
                              const float* gy, const double* step_beta, void* stream);

/* The schedule of one Nesterov iteration on the device (Section IV-A: the
 * step interval, the gamma rule and the lambda update), so that a loop of
 * fftpl_eval_params, fftpl_step_stats, fftpl_nesterov_schedule and
 * fftpl_nesterov_update_dev needs no host read per iteration.  One thread
 * reads stats (device double[4], fftpl_step_stats' out4) and out4 (device
 * double[4], the evaluation's [N, W~, HPWL, tau]) and updates state (device
 * double[FFTPL_LOOP_STATE]):
 *   [0] a (Nesterov sequence), [1] alpha_max, [2] alpha_min (physical units),
 *   [3] lambda, [4] gamma, [5] k (iterations done), [6] the previous
 *   iteration's HPWL (NaN: none), [7] alpha_max_0, [8] bin width,
 *   [9] lambda rule (0: doubled every [10] iterations, and a restarts at 1
 *   when [11] != 0; 1: the paper's mu_k = 1.1^(1 - dHPWL / 3.5e5) bounded to
 *   [0.75, 1.1]), [12], [13] (out) step and beta of this iteration's update,
 *   [14] the first logged k.
 * This iteration: alpha = the Barzilai-Borwein estimate sqrt(stats[0] /
 * stats[1]) * stats[2] kept in [alpha_min, alpha_max] (alpha_max at k = 0 or
 * when either sum is 0), step = alpha / stats[2] (0 when stats[2] = 0),
 * a' = (1 + sqrt(4 a^2 + 1)) / 2, beta = (a - 1) / a'.  Next iteration:
 * alpha_max = max(alpha_max_0, 2 alpha), alpha_min = 0.01 alpha_max,
 * gamma = 8 bin 10^(20/9 (tau - 0.1) - 1), lambda by the rule, and params
 * (device float[2]) = (lambda, gamma) for fftpl_eval_params.  If
 * 0 <= k - state[14] < log_cap, log[8 (k - state[14]) + 0..7] = [k, N, W~,
 * HPWL, tau, lambda, gamma, alpha] with this iteration's values (log: device
 * double[8 log_cap], may be NULL when log_cap = 0).  Double arithmetic in the
 * host rule's order. */
#define FFTPL_LOOP_STATE 16
int fftpl_nesterov_schedule(const double* stats, const double* out4, double* state,
                            float* params, double* log, int32_t log_cap, void* stream);

/* Nonlinear conjugate gradients, the inner solver of Algorithm 1 (the
 * "CGsolver" step: one direction and one line search inside the step
 * interval [alpha_min, alpha_max] of Section IV-A per outer iteration).  The
 * direction update and the line search are chosen on the host from these
 * device reductions (all double, over both axes of num_cells cells,
 * per-block partials summed in a fixed order):
 *   fftpl_cg_dots:      out4 = [g.g, g.gp, gp.gp, g.d] (gp, gpx/gpy the previous
 *                       gradient, d the previous direction; either pair may be
 *                       NULL: its terms are 0);
 *   fftpl_cg_direction: d = -g + beta d (beta >= 0; beta = 0 restarts with
 *                       d = -g and does not read d), *dmax = max |d| over the
 *                       components (a device double);
 *   fftpl_cg_move:      xo = clamp(x + t d) per axis, with clamp keeping each
 *                       cell (sizes w, h) inside the region of `region` (as
 *                       fftpl_nesterov_update); xo, yo may alias x, y.
 * work: device double scratch of at least 1024 entries (work_doubles). */
int fftpl_cg_dots(int32_t num_cells, const float* gx, const float* gy, const float* gpx,
                  const float* gpy, const float* dx, const float* dy, double* out4,
                  double* work, uint64_t work_doubles, void* stream);
int fftpl_cg_direction(int32_t num_cells, const float* gx, const float* gy, float beta,
                       float* dx, float* dy, double* dmax, double* work, uint64_t work_doubles,
                       void* stream);
int fftpl_cg_move(const fftpl_grid* region, int32_t num_cells, const float* w, const float* h,
                  const float* x, const float* y, const float* dx, const float* dy, float t,
                  float* xo, float* yo, void* stream);

/* Test export: the integer bin range of every cell under the rectangle rule
 * above, ranges[4*i + {0,1,2,3}] = {ix0, ix1, iy0, iy1} (empty when first >
 * last).  ranges is a device int32 array [4*num_cells]. */
int fftpl_debug_cell_bins(const fftpl_grid* grid, int32_t num_cells, const float* x,
                          const float* y, const float* w, const float* h,
                          int32_t* ranges, void* stream);

/* Test export: per-net values as the exchange path computes them (Eqs. (1),
 * (3), or the log-sum-exp model per prob->wl_model), for a problem with an
 * exchange index and workspace: for every net e with at least one pin,
 * wl_first[net_ptr[e]] = its wirelength term over both axes and
 * hpwl_first[net_ptr[e]] = its half-perimeter; device double arrays
 * [num_pins] whose other entries are left as they are.  Errors as for
 * fftpl_problem_wl_grad. */
int fftpl_debug_net_values(const fftpl_problem* prob, const float* x, const float* y,
                           float gamma, double* wl_first, double* hpwl_first, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FFTPL_H */
