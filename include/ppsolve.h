/*
 * ppsolve — FFT + Thomas direct solve of the second-order 7-point Poisson
 * problem on one AMD MI355X (gfx950).
 *
 * Method: PittPack, Hasbestan & Senocak, arXiv:1909.05423.  The discrete
 * problem is the cell-centred 7-point stencil of section "Mathematical
 * Formulation" (Eq. 3) on a directionally uniform grid, with periodic,
 * homogeneous Dirichlet or homogeneous Neumann faces (section "Boundary
 * Conditions").  The solve applies the forward real transforms along x and y
 * (periodic -> DFT, Neumann -> DCT-II, Dirichlet -> DST-II; Table
 * TransformationList), one tridiagonal solve along z per wavenumber pair with
 * the modified wavenumbers of Table eig (section "Solution of the Resulting
 * Tridiagonal Matrices", Algorithm Thomas for Toeplitz Matrices), and the
 * inverse transforms.  The singular zero mode of pure Neumann/periodic problems
 * is pinned (section "Well-posedness").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Arrays are C-contiguous (batch, nz, ny, nx), x fastest, in device memory.
 * Cell (i, j, k) sits at ((i + 1/2) hx, (j + 1/2) hy, (k + 1/2) hz).
 * The equation is  sum_d (u_{+1} - 2 u + u_{-1}) / h_d^2 = f  (no minus sign).
 * The caller owns f, u and the workspace; a plan owns only host memory.
 * Every launch goes on the caller's HIP stream (`stream` is a hipStream_t;
 * NULL is the default stream) and the calls return before the GPU work ends,
 * except the refined mode, which reads one pair of scalars back per
 * refinement step.  No status crosses the ABI as an exception.
 */
#ifndef PPSOLVE_H
#define PPSOLVE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_plan_s* pp_plan;

/* Arithmetic of a plan.
 *   PP_F64          f, u are double; transforms and z-solves in double.
 *   PP_F32          f, u are float; transforms and z-solves in float.
 *   PP_F32_REFINED  f, u are double; every solve runs in float (save the x
 *                   transform's arithmetic and the lowest x-wavenumber slots,
 *                   see pp_plan_set_refinement), wrapped in iterative
 *                   refinement whose residual (the 7-point stencil of Eq. 3
 *                   with the face ghost rules) and solution update are
 *                   accumulated in double on the GPU. */
typedef enum { PP_F64 = 0, PP_F32 = 1, PP_F32_REFINED = 2 } pp_dtype;

/* Treatment of the singular zero mode (pure Neumann/periodic x and y with
 * Neumann or periodic z faces); ignored for non-singular problems.
 *   PP_GAUGE_MEAN     subtract the volume mean of f (the alternative the
 *                     "Well-posedness" section names), pin, then shift u to
 *                     zero volume mean.  Unique; the solve operator is symmetric.
 *   PP_GAUGE_PIN      subtract the mean of f and pin: the first unknown of the
 *                     (kx, ky) = (0, 0) z-system is zero, i.e. the mean of u over
 *                     the first z plane is zero (the paper's default pin).
 *   PP_GAUGE_PIN_RAW  pin only, no projection: the plane z = 0 absorbs the
 *                     incompatible part of f. */
typedef enum { PP_GAUGE_MEAN = 0, PP_GAUGE_PIN = 1, PP_GAUGE_PIN_RAW = 2 } pp_gauge;

typedef enum {
    PP_OK = 0,
    PP_ERR_ARG = -1,           /* null pointer, non-positive size/spacing/batch, bad enum */
    PP_ERR_BC = -2,            /* bc char not in {P,D,N}; x or y faces of different types;
                                  one z face periodic and the other not */
    PP_ERR_SIZE = -3,          /* nx or ny has a prime factor other than 2 and 3, or exceeds
                                  the on-chip line limit (2048), or nz * batch > 65535 */
    PP_ERR_ALIAS = -4,         /* u (or out) overlaps f (or g) or the workspace */
    PP_ERR_WORKSPACE = -5,     /* workspace pointer null or misaligned (256 B) */
    PP_ERR_HIP = -6,           /* a HIP call failed (launch, copy, synchronisation) */
    PP_ERR_NOT_CONVERGED = -7, /* refinement did not reach its tolerance in max_iter steps */
    PP_ERR_NONFINITE = -8,     /* the source held an Inf or NaN (reported where the
                                  library reads scalars back: refinement, last_info) */
    PP_ERR_SCRATCH = -9        /* pp_solve_noalloc: the plan needs more workspace than
                                  PP_NOALLOC_SCRATCH_BYTES */
} pp_status;

/* Limits (the plan call returns PP_ERR_SIZE beyond them):
 *   nx, ny      factor as 2^a 3^b and are at most 2048 (whole lines are held on
 *               chip; y lines up to 1024 take the pipelined z march, longer ones
 *               a slower general march);
 *   nz * batch  at most 65535 (launch grid of the refinement residual);
 *   periodic z  nz >= 3;
 *   PCR / CR-P  z not periodic (PP_ERR_BC), nz at most 4096 and ny at most 512
 *               (set_zsolver).
 * Device workspace: pp_plan_workspace_bytes(p); about 8 B (PP_F64, and
 * PP_F32_REFINED; 16 B with rows over 512) or 4 B (PP_F32) per grid point and
 * batch entry, plus the plan tables (and, for the split march below, two
 * values per (x-wavenumber slot, y entry, batch entry), for the segmented
 * march four per (slot, y entry, batch entry, segment)). */

/* Create a plan (host only; no GPU call).
 *   nx, ny, nz  cells per direction, >= 1.  nx and ny must factor as 2^a 3^b.
 *   bc          6 chars for the faces (x-, x+, y-, y+, z-, z+) from
 *               'P' periodic, 'D' homogeneous Dirichlet (value 0 on the face,
 *               ghost cell by linear extrapolation), 'N' homogeneous Neumann
 *               (zero flux).  The two x faces share a type, as do the two y
 *               faces (Table eig lists only PP, NN, DD); z faces are D or N,
 *               each independently, or both P (periodic z: each z-system is
 *               cyclic and is solved through the Sherman-Morrison splitting of
 *               the Thomas subsection; needs nz >= 3, else PP_ERR_SIZE).
 *   h           spacings (hx, hy, hz) > 0.
 *   dtype       see pp_dtype.  batch: independent right-hand sides, >= 1.
 * On success *out holds a plan to release with pp_plan_destroy.  The gauge
 * defaults to PP_GAUGE_MEAN; refinement to tol 1e-13 (estimated relative
 * error), max_iter 8. */
pp_status pp_plan_create(int nx, int ny, int nz, const char bc[6], const double h[3],
                         pp_dtype dtype, int batch, pp_plan* out);

/* Select the zero-mode treatment (see pp_gauge). */
pp_status pp_plan_set_gauge(pp_plan p, pp_gauge gauge);

/* z solver (sections "Solution of the Resulting Tridiagonal Matrices",
 * "Cyclic Reduction Technique", "Parallel Cyclic Reduction").
 *   PP_ZSOLVER_THOMAS  default: Thomas, fused with the y transforms in one
 *                      march along z (two passes over the spectral array).
 *                      Non-periodic z with few columns (see pp_zsplit) splits
 *                      each z-system at a point near its middle: the upper
 *                      part is eliminated from z = 0 and the lower part from
 *                      z = nz-1 by two workgroups, which then solve the two
 *                      meeting rows and substitute outward (same passes).
 *   PP_ZSOLVER_PCR     parallel cyclic reduction on whole z lines in LDS, with
 *                      the y transforms as separate passes (four passes);
 *   PP_ZSOLVER_CR      cyclic reduction with a parallel backward phase (CR-P),
 *                      arranged like PCR.
 *   PCR and CR-P: nz <= 4096 and ny <= 512 (PP_ERR_SIZE otherwise), z not
 *   periodic (PP_ERR_BC).  For comparison with the default. */
typedef enum { PP_ZSOLVER_THOMAS = 0, PP_ZSOLVER_PCR = 1, PP_ZSOLVER_CR = 2 } pp_zsolver;
pp_status pp_plan_set_zsolver(pp_plan p, pp_zsolver solver);

/* Layout of the Thomas march (PP_ZSOLVER_THOMAS; the other solvers ignore it).
 *   PP_ZSPLIT_AUTO  default: split where the columns (x-wavenumber slots times
 *                   batch) are at most 1/2 (PP_F64), 2 (PP_F32) or 4
 *                   (PP_F32_REFINED) per compute unit of the device, or, in
 *                   PP_F64 on y lines up to 512 with more columns than
 *                   compute units, where the split's rounds of workgroups
 *                   (two launches of ceil(2 columns / CUs), each about a
 *                   quarter of a column's march) take less than the whole
 *                   march's ceil(columns / CUs); and, in place of either,
 *                   segmented wherever the plan has segments (below), provided
 *                   no z-system is so close to singular that splitting it
 *                   amplifies rounding by more than 256 (the zero mode and
 *                   lowest wavenumbers of long columns under Neumann or
 *                   periodic x, y faces: about nz / 2 for the zero mode).
 *                   That bound keeps PP_F64 plans to one march per column;
 *                   PP_F32 and PP_F32_REFINED plans keep the two-way split
 *                   (float rounding dominates its error) and drop only the
 *                   segments;
 *   PP_ZSPLIT_OFF   always one workgroup per column;
 *   PP_ZSPLIT_ON    always split in two (two workgroups per column);
 *   PP_ZSPLIT_SEG   always segmented: each column in 3 to 16 segments, each
 *                   eliminated on its own, their end rows coupled through a
 *                   small reduced system solved between two launches.
 *                   Segments enough for about 256 workgroups on y lines over
 *                   256, 768 (PP_F64) or 1024 (PP_F32) on lines up to 256;
 *                   the form exists for f64 and f32 plans where that means
 *                   three segments or more (columns at most 85 on lines over
 *                   256; 256 in f64, 341 in f32 on lines up to 256) and nz
 *                   holds three segments of at least two chunks.
 * The split form exists for non-periodic z, y lines up to 1024 and nz of at
 * least two chunks of the march (16 planes; 12 for float lines of 384, 8 for
 * double lines over 512): PP_ZSPLIT_ON / PP_ZSPLIT_SEG on other shapes return
 * PP_ERR_BC (periodic z) or PP_ERR_SIZE.  All layouts solve the same
 * z-systems; forced splits of near-singular systems carry errors up to about
 * the amplification above times the unit roundoff (measured: 1.3e-12
 * relative for the two-way split and 3e-12 segmented at 16 x 16 x 1023 with
 * Neumann z and periodic x, y, against 3.5e-15 for one march; in PP_F32
 * 8e-7 split and 3.7e-5 segmented against 1.5e-6). */
typedef enum { PP_ZSPLIT_AUTO = 0, PP_ZSPLIT_OFF = 1, PP_ZSPLIT_ON = 2, PP_ZSPLIT_SEG = 3 } pp_zsplit;
pp_status pp_plan_set_zsplit(pp_plan p, pp_zsplit mode);

/* Refinement controls for PP_F32_REFINED: stop once the estimated relative
 * error of u (max-norm) is at most tol, or after max_iter correction steps
 * (max_iter = 0 runs the float solve alone and reports PP_ERR_NOT_CONVERGED).
 * The estimate is the size of the next correction: the last correction times
 * the ratio of the last two corrections, or, after the first, times the first
 * correction itself (the float solve's relative error, which the correction's
 * solve is taken to repeat).  The float solves transform along x in double and
 * keep the spectra of the 16 lowest x-wavenumber slots in double through the
 * z march (y lines up to 1024; on longer lines those slots run in float too
 * and more corrections may be needed). */
pp_status pp_plan_set_refinement(pp_plan p, double tol, int max_iter);

/* Bytes of device workspace the caller must pass to pp_solve/pp_solve_adjoint
 * (256-byte aligned).  0 for a null plan. */
size_t pp_plan_workspace_bytes(pp_plan p);

/* Solve L_h u = f for every batch entry.  f and u: device arrays of
 * batch*nz*ny*nx doubles (PP_F64, PP_F32_REFINED) or floats (PP_F32); they
 * must not overlap each other or the workspace.  f is read only.
 * Workspace ownership: the library records, per workspace base pointer, which
 * plan last uploaded its tables there.  A call with a workspace that this plan
 * did not fill last uploads the plan's tables into it (an asynchronous copy on
 * `stream`); later calls reuse them.  So several plans may share one workspace
 * (each call then re-uploads when the previous one was another plan's), but
 * the caller must not write into a workspace between solves, must not pass
 * workspaces of different plans that overlap without starting at the same
 * address, and must not free a workspace and hand a new allocation at the same
 * address to the plan that used the old one (its tables would be taken as
 * present).  The Python binding allocates one workspace per plan and holds it
 * for the plan's lifetime. */
pp_status pp_solve(pp_plan p, const void* f, void* u, void* workspace, void* stream);

/* Solve with non-homogeneous face values (section "Boundary Conditions":
 * the part of each ghost value that does not depend on u moves to the
 * right-hand side, so the boundary cells of a Dirichlet face solve with
 * f - 2 g / h^2 and those of a Neumann face with f - g / h).
 *   faces  array of 6 device pointers in the order x-, x+, y-, y+, z-, z+; each
 *          is NULL (homogeneous face) or holds, per batch entry, the face's
 *          values in C order: x faces [batch][nz][ny], y faces [batch][nz][nx],
 *          z faces [batch][ny][nx], in the element type of f.  A Dirichlet face
 *          carries the value of u on the face; a Neumann face the derivative of
 *          u along the outward normal.  A periodic face must be NULL.
 * faces itself may be NULL (same as pp_solve).  Face arrays are read only and
 * must not overlap u or the workspace.  Otherwise as pp_solve.  In a singular
 * problem the compatibility projection removes the mean of the lifted source,
 * so Neumann fluxes and f need not balance.
 * Errors: PP_ERR_ARG for a value on a periodic face or a misaligned face
 * pointer; PP_ERR_ALIAS for a face overlapping u or the workspace. */
pp_status pp_solve_bc(pp_plan p, const void* f, const void* const faces[6], void* u, void* workspace, void* stream);

/* out = G^T g, the transpose of the linear map f -> u that pp_solve applies,
 * for dJ/df = G^T dJ/du.  Same array rules as pp_solve.  The transforms, the
 * z-systems (symmetric: equal off-diagonals) and the per-mode weights of the
 * real-data transforms transpose into the same stage sequence as the forward
 * solve; what changes is the zero-mode treatment, whose projection and mean
 * shift trade places (PP_GAUGE_PIN: pin, then subtract the mean of the
 * result). */
pp_status pp_solve_adjoint(pp_plan p, const void* g, void* out, void* workspace, void* stream);

/* Results of the last pp_solve/pp_solve_adjoint on this plan; synchronises
 * with that call's stream.  Any pointer may be NULL.
 *   ir_iters          refinement corrections applied (0 unless PP_F32_REFINED)
 *   removed_mean      array of `batch` doubles: volume mean of the source that
 *                     the projection removed (0 where nothing was removed)
 *   final_rel_update  last ||correction||_inf / ||u||_inf (refined mode)
 * Returns PP_ERR_NONFINITE when the last source held an Inf or NaN. */
pp_status pp_plan_last_info(pp_plan p, int* ir_iters, double* removed_mean, double* final_rel_update);

/* Kernel timing (off by default).  With timing on, every solve records HIP
 * events on its stream around each kernel launch.  pp_plan_kernel_times
 * synchronises with the recorded events and returns, for the kernel groups
 *   0 x forward (transform + transpose), 1 z march (y transforms + z solves),
 *   2 x inverse, 3 everything else (reductions, residual, refinement control),
 * the accumulated milliseconds and launch counts since the last reset
 * (arrays of 4; either may be NULL); reset != 0 clears the accumulators. */
pp_status pp_plan_set_timing(pp_plan p, int on);
pp_status pp_plan_kernel_times(pp_plan p, double* ms, int* launches, int reset);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * pp_solve with the workspace replaced by a fixed buffer of
 * PP_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * (from the first use until the process ends).  Calls no allocator.  Same f, u,
 * stream and error rules as pp_solve (face values and the adjoint are not
 * offered here), plus PP_ERR_SCRATCH when pp_plan_workspace_bytes(p) exceeds
 * the buffer.  Every call on one device shares that device's buffer: calls
 * that overlap in time on one device (other streams, other threads) race and
 * must be ordered by the caller.  The first call of a plan after another plan
 * used the buffer copies the plan's tables into it from host memory (so a
 * caller capturing a graph makes one call before the capture). */
#define PP_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
pp_status pp_solve_noalloc(pp_plan p, const void* f, void* u, void* stream);

/* Measurement utility, not part of the solve: copies `bytes` (a multiple of 16;
 * src and dst 16-byte aligned, not overlapping) between device buffers with
 * 16-byte non-temporal loads and stores over a persistent grid, on `stream`.
 * Every kernel of the solve streams its input once and its output once, so the
 * bandwidth of this copy is the practical ceiling their achieved bandwidth is
 * compared with.  PP_ERR_ARG / PP_ERR_ALIAS / PP_ERR_HIP. */
pp_status pp_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

void pp_plan_destroy(pp_plan p);

/* Static, NUL-terminated description of a status code. */
const char* pp_status_string(pp_status st);

#ifdef __cplusplus
}
#endif

#endif /* PPSOLVE_H */
