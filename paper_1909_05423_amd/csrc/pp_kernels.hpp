// Kernel argument blocks and host launchers shared by the plan code and the
// kernel sources.  Internal to the library: the public ABI is include/ppsolve.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

#include "pp_device.hpp"
#include "../../include/ppsolve.h"

namespace pp {

enum Bc : int { BC_P = 0, BC_N = 1, BC_D = 2 };

// Launch shapes.  Every transform kernel gives each thread at most kEpt
// complex values of the lines it holds in LDS (FFT stages keep one radix-8
// butterfly, two radix-4, three radix-3 or four radix-2 butterflies per thread
// in registers).
constexpr int kEpt = 8;
constexpr int kXThreads = 256;                 // x kernels: lines of nx per workgroup = kXElems / nx
constexpr int kXElems = kXThreads * kEpt;
constexpr int kXBlocksPerCU = 2;               // persistent x-kernel workgroups per CU (all resident)
constexpr int kXWaves = kXThreads / 64;
constexpr int kXLdsBytes = 96 * 1024;          // x-kernel LDS target (lines + twiddle tables), two workgroups per CU
constexpr int kXLdsMax = 160 * 1024 - 1024;    // x-kernel LDS ceiling (one workgroup per CU)
// x-kernel register shape: values per lane of one line (64 * RMAX >= nx).
constexpr int xdir_rmax(int nx) { return nx <= 512 ? 8 : (nx <= 1024 ? 16 : 32); }
constexpr int kZThreads = 512;                 // z march: planes per chunk = kZElems / ny
constexpr int kZElems = kZThreads * kEpt;
// Entries (spectral y positions) one thread of the z march owns: ny <= kZThreads * kZOwned;
// a chunk holds zb <= kEpt / ceil(ny / kZThreads) planes.
constexpr int kZOwned = 4;
constexpr int kMaxLine = 2048;                 // longest x or y line
// z-march LDS budget: zb padded lines plus ny twiddles.
constexpr int kZLdsBytes = 160 * 1024 - 1024;
constexpr size_t zmarch_lds_bytes(int zb, int ldy, int ny, size_t elem) {
    return ((size_t)zb * ldy + (size_t)ny) * elem;
}
// z-march register shape: values per lane of a chunk (64 * RMAX >= ny).
constexpr int zmarch_rmax(int ny) { return ny <= 512 ? 8 : (ny <= 1024 ? 16 : 32); }

// x-direction kernels: a workgroup owns `ty` consecutive rows (y0 .. y0+ty-1)
// of one z plane of one batch entry, packed two rows per complex line.
template <typename T> struct XArgs {
    int nx, ny, nz, slots;   // slots = ceil(nx/2) spectral columns per row
    int bx;                  // boundary type along x (Bc)
    int ty;                  // rows per workgroup (even; ty/2 * nx <= kXElems)
    int ldl;                 // LDS line stride (padded_len(nx))
    long sstride, zstride;   // spectral array: element (b, m, z, y) at b*slots*nz*ny + m*sstride + z*zstride + y
    FftDesc fx;              // radix plan for nx
    const cplx<T>* twx;      // FFT twiddles of length nx, packed by stage (wfft_stage)
    const cplx<T>* mkx;      // exp(-i pi k / (2 nx)), k < nx
    // split store of the forward kernel (double arithmetic, float spectra): slots
    // lo0 .. lo0+nlo-1 go to the double array slo [b][z][k][y] instead
    int lo0, nlo;
    cplx<double>* slo;
    // fused refinement residual (forward kernel with RES): the rows transformed
    // are r = f - lift - c - L_h u0 (double arithmetic; c as in ResidualArgs),
    // and the spectra are stored scaled by sc[SC_SCALE]
    const float* u0;
    const double* sc;
    int fbc[6];              // face types (Bc), x-, x+, y-, y+, z-, z+
    int proj;
    double ihx2, ihy2, ihz2;
    // inverse kernels: take the z planes of each batch entry from both ends
    // inward (0, nz-1, 1, nz-2, ...), the order in which the split z march
    // finishes them, so that the most recently written planes are read first
    int zends;
};

// Non-homogeneous face values, faces in the order x-, x+, y-, y+, z-, z+.  The
// part of a ghost value that does not depend on u moves to the right-hand side
// (section "Boundary Conditions"): the boundary cells of face i take
// f - c_i g_i, with c = 2/h^2 for a Dirichlet value g and 1/h for a Neumann
// outward derivative g.  g[i] is null for a homogeneous or periodic face.
// Layout per batch entry (C order): x faces [nz][ny], y faces [nz][nx],
// z faces [ny][nx].
template <typename Tin> struct FaceArgs {
    const Tin* g[6];
    double c[6];
};

// Lift of the y and z face values at cell (i, j, k) of batch entry b (zero off those faces).
template <typename Tin>
__device__ __forceinline__ double face_lift_yz(const FaceArgs<Tin>& fa, int b, int i, int j, int k, int nx, int ny,
                                               int nz) {
    double l = 0.0;
    if (j == 0 && fa.g[2]) l += fa.c[2] * (double)fa.g[2][((size_t)b * nz + k) * nx + i];
    if (j == ny - 1 && fa.g[3]) l += fa.c[3] * (double)fa.g[3][((size_t)b * nz + k) * nx + i];
    if (k == 0 && fa.g[4]) l += fa.c[4] * (double)fa.g[4][((size_t)b * ny + j) * nx + i];
    if (k == nz - 1 && fa.g[5]) l += fa.c[5] * (double)fa.g[5][((size_t)b * ny + j) * nx + i];
    return l;
}

// Lift of all face values at cell (i, j, k) of batch entry b (zero off the faces).
template <typename Tin>
__device__ __forceinline__ double face_lift(const FaceArgs<Tin>& fa, int b, int i, int j, int k, int nx, int ny,
                                            int nz) {
    double l = face_lift_yz(fa, b, i, j, k, nx, ny, nz);
    if (i == 0 && fa.g[0]) l += fa.c[0] * (double)fa.g[0][((size_t)b * nz + k) * ny + j];
    if (i == nx - 1 && fa.g[1]) l += fa.c[1] * (double)fa.g[1][((size_t)b * nz + k) * ny + j];
    return l;
}

// Solution mode of the inverse x kernel.
// XINV_UPDATE adds the correction to u; XINV_FIRST stores the first solution
// of the refinement without reading u.
enum XinvMode : int { XINV_STORE = 0, XINV_UPDATE = 1, XINV_FIRST = 2 };

// segmented z march: at most this many segments per column (the reduced
// system's kernel keeps one row per segment in registers)
constexpr int kMaxZSegments = 16;

// z-march kernel: one workgroup per (spectral x column, batch entry).
template <typename T> struct MidArgs {
    int ny, nz, slots;
    int bx, by;
    int ldy;                 // LDS line stride (padded_len(ny))
    int zb;                  // z planes per LDS chunk (zb * ny <= kZElems, zb * own <= kEpt)
    int singular;            // zero mode present (slot 0, entry 0, real part)
    int project;             // subtract the source mean from the zero-mode line
    int demean;              // report the mean of the zero-mode solution (subtracted by the x inverse)
    long sstride, zstride;   // spectral array strides (as in XArgs)
    T scale;                 // hz^2 / (nx ny): all transform normalisations and the z-system scaling
    double hz2;              // hz^2 (projection constant = hz^2 * mean(f))
    FftDesc fy;
    const cplx<T>* twy;      // FFT twiddles of length ny, packed by stage (wfft_stage)
    const cplx<T>* mky;      // exp(-i pi k / (2 ny))
    const int* rowoff;       // per slot: first table row
    const int* lmax;         // per slot: rows stored (z < lmax reads the table)
    const int* elen;         // per (slot, entry): rows in which this entry's pivots differ from winf (<= lmax)
    const cplx<T>* wrows;    // [row][ny] (w_re, w_im) reciprocal pivots
    const cplx<T>* winf;     // [slot][ny] converged reciprocal pivot
    const cplx<T>* wlast;    // [slot][ny] reciprocal pivot of the last row
    // split march (non-periodic z): rows 0 .. zsplit-1 eliminated downward from
    // z = 0 with the pivots above, rows zsplit .. nz-1 upward from z = nz-1 with
    // the pivots of the reversed system (row nz-1-j at table row j); the two
    // halves meet between rows zsplit-1 and zsplit.  zsplit 0: one march.
    int zsplit;
    const int* browoff;      // as rowoff / elen / wrows / winf, for the lower half
    const int* belen;
    const cplx<T>* bwrows;
    const cplx<T>* bwinf;
    const cplx<T>* meet;     // [slot][ny][3]: w of row zsplit-1, v of row zsplit, 1 / (1 - v w)
    cplx<T>* zbuf;           // [batch][slot][2][ny]: last eliminated value of each half
    // segmented march (zsegs >= 3): segment s holds rows [s zseglen, ...), the
    // last one the remainder; each segment eliminated on its own (fresh
    // pivots outside segment 0, the last row of the last segment with the
    // bottom face), its couplings to the neighbouring segments solved from the
    // segments' end values, then applied on the way back
    int zsegs, zseglen;
    const int* frowoff;      // fresh pivots, as rowoff / elen / wrows / winf
    const int* felen;
    const cplx<T>* fwrows;
    const cplx<T>* fwinf;
    const cplx<T>* flast;    // [slot][ny] last row of the last segment
    const int* rrowoff;      // rho (fresh elimination of a segment's first unit vector) rows
    const int* relen;
    const cplx<T>* rrows;
    const cplx<T>* rholast;  // [slot][ny] rho at the last row of the last segment
    const cplx<T>* segk;     // [slot][ny][3 classes][4]: p_first, p_last, q_first, q_last
    cplx<T>* segg;           // [batch][slot][zsegs][2][ny]: segment end values (local solution)
    cplx<T>* seglr;          // [batch][slot][zsegs][2][ny]: couplings above / below each segment
    // periodic z (Sherman-Morrison, see the plan code): per slot, rows of
    // alpha = first row of the inverse of the split matrix and of the
    // forward-eliminated rank-one vector; per entry its last value, 1/den, 1/gamma
    int zper;
    const int *aoff, *alen, *qoff, *qlen;
    const int *aelen, *qelen;   // per (slot, entry): rows of alpha / qp before they are zero
    const cplx<T> *arows, *qrows, *qlast, *inv_den, *inv_gamma;
    // z solver: 0 = fused Thomas march, 1 = parallel cyclic reduction, 2 = CR-P (separate y passes)
    int zsolver;
    int bz0, bz1;            // z face types (Bc) of the end rows
    const cplx<T>* bmid;     // [slot][ny] interior diagonal hz^2 lam - 2 of each part's z-system
    const double* mu;        // [batch] source means
    double* cmean;           // [batch] mean of the zero-mode solution line (output)
};

// IR residual r = scale * (f - c - L_h u) in float, where c is the part of f
// outside the range of L_h in a singular problem (known from the source mean):
//   proj 0: none (non-singular); 1: mean(f) everywhere (projected gauges);
//   2: nz * mean(f) on the plane z = 0 only (pinned gauge without projection).
struct ResidualArgs {
    int nx, ny, nz, batch;
    int bc[6];
    int proj;
    double ihx2, ihy2, ihz2;
    FaceArgs<double> faces;  // non-homogeneous face values (all null: homogeneous)
    int has_faces;
};

// --- launchers (return hipError_t of the launch) -----------------------------
// Row blocks of the x kernels and the persistent grid they run on; the x kernels
// write one partial record per (batch entry, workgroup, wavefront).
int x_blocks(int ny, int ty, int nz, int batch);
int x_grid(int nblocks);
// Grid of an x-kernel launch over nblocks row blocks: when the workgroups take
// blocks in pairs (the inverse kernel with float spectra, x_next_block), half
// as many are needed.
int x_launch_grid(int nblocks, bool paired);

// faces: null, or the face values to lift into the source as it is read.
// T: arithmetic; Tin: source; Ts: spectra (T, or float with the double slots of XArgs::slo).
template <typename T, typename Tin, typename Ts>
hipError_t launch_xfwd(const Tin* f, cplx<Ts>* S, double* partial, const XArgs<T>& a, int batch,
                       const FaceArgs<Tin>* faces, hipStream_t s);
// The forward transform of the refinement residual r = f - lift - c - L_h u0
// (XArgs::u0, sc, fbc, proj, ih*2), computed as the rows are read: double
// arithmetic, float spectra with the double slots.  Rows of at most 512
// (res_fused_supported); other shapes take launch_residual + launch_xfwd.
bool res_fused_supported(int nx);
hipError_t launch_xfwd_res(const double* f, cplx<float>* S, double* partial, const XArgs<double>& a, int batch,
                           const FaceArgs<double>* faces, hipStream_t s);

template <typename T, typename Tout>
hipError_t launch_xinv(const cplx<T>* S, Tout* u, const XArgs<T>& a, int batch, const double* shift,
                       hipStream_t s);

// Refinement updates, with partials (sum over the gauge region of the new u,
// max |d / scale|, max |u_new|) per wavefront.
//   launch_xinv_first:  u0 = d / scale, stored in float (the first solve; its
//                       float values unshifted, so the store rounds nothing);
//   launch_xinv_update: mode XINV_FIRST: u = d / scale - cmean (double);
//                       XINV_UPDATE: u = prev + d / scale - cmean - gauge_shift[b],
//                       prev = uprev (float) when given, else u itself.
hipError_t launch_xinv_first(const cplx<float>* S, float* u0, const XArgs<float>& a, int batch, const double* scalars,
                             int gauge_region, double* partial, hipStream_t s);
hipError_t launch_xinv_update(const cplx<float>* S, double* u, const float* uprev, const XArgs<float>& a, int batch,
                              const double* scalars, int gauge_region, double* partial, int mode, hipStream_t s);

template <typename T>
hipError_t launch_mid(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s);

// Compute units of the current device (256 if the query fails).
int device_cus();
// Raise a kernel's dynamic-LDS limit to `bytes` on the current device, once
// per (kernel, device) and thread-safe; returns the error of the attribute
// call (hipSuccess when already set).
hipError_t allow_dynamic_lds(const void* kernel, int bytes);
// Planes per chunk of the pipelined z march for lines of ny in double or float
// (0: no pipelined form, ny over 1024); the split march puts its meeting
// point on a multiple of it.
int zpipe_planes(int ny, bool dbl);

// The refined solve's z stage: slots lo0 .. lo0+nlo-1 from their double
// spectra Slo in double (tables of ad), the rest in float (tables of af); every
// result in float in S.  Supported where mixed_march_supported().
bool mixed_march_supported(int ny, int zsolver);
hipError_t launch_mid_mixed(const cplx<double>* Slo, cplx<float>* S, const MidArgs<double>& ad,
                            const MidArgs<float>& af, int lo0, int nlo, int batch, hipStream_t s);

// The same stage with the z-systems solved by parallel cyclic reduction
// (y transforms as separate passes; nz <= 512, ny <= 512, z not periodic).
template <typename T>
hipError_t launch_mid_pcr(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s, bool cr);

// Finalise the x-forward partials: mu[b] = sum / npts, scalars[SC_MAXF] = max |f|.
hipError_t launch_finalize_xfwd(const double* partial, int nper, int batch, double npts, double* mu,
                                double* maxf, hipStream_t s);

// Finalise the refinement-update partials into the scalar block and choose the
// next residual scale.
hipError_t launch_finalize_update(const double* partial, int nper, int batch, double nregion, double* scalars,
                                  int first, hipStream_t s);

template <typename Tu, typename Tr>
hipError_t launch_residual(const double* f, const Tu* u, Tr* r, const ResidualArgs& a,
                           const double* scalars, hipStream_t s);

// Streaming device copy of `bytes` (a multiple of 16), the bandwidth reference.
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// Initial scalars of the refinement loop (unit scale, no gauge shift).
hipError_t launch_ir_init(double* scalars, int batch, hipStream_t s);

// Fixed workspace of pp_solve_noalloc (one per device, inside the library).
constexpr size_t kScratchBytes = (size_t)PP_NOALLOC_SCRATCH_BYTES;
// Device address of this device's fixed workspace (looked up once per device).
hipError_t scratch_buffer(void** ptr);

// Scalar block layout (doubles) used by the refinement loop.
enum Scalar : int {
    SC_MAXF = 0,      // max |f|
    SC_MAXD = 1,      // max |correction| of the last update
    SC_MAXU = 2,      // max |u| after the last update
    SC_REL = 3,       // SC_MAXD / SC_MAXU
    SC_RELPREV = 4,   // previous SC_REL
    SC_SCALE = 5,     // residual scale of the current step (power of two)
    SC_INVSCALE = 6,  // 1 / SC_SCALE
    SC_COUNT = 16     // per-batch arrays follow
};

}  // namespace pp
