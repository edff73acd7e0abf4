// Small kernels around the solve: reductions of per-workgroup partials, the
// double-precision 7-point residual of the refinement loop and its control
// scalars.

#include <cmath>

#include "pp_kernels.hpp"

namespace pp {

constexpr int kRedThreads = 1024;

// One workgroup: per batch entry, the sum of the (sum, max) pairs written by
// the forward x kernel, in a fixed order (deterministic).
__global__ __launch_bounds__(kRedThreads) void k_finalize_xfwd(const double* __restrict__ partial, int nper,
                                                               int batch, double npts, double* __restrict__ mu,
                                                               double* __restrict__ maxf) {
    __shared__ double red[kRedThreads / 64];
    double gmax = 0.0;
    for (int b = 0; b < batch; ++b) {
        double s = 0.0, mx = 0.0;
        for (int i = threadIdx.x; i < nper; i += kRedThreads) {
            s += partial[2 * ((size_t)b * nper + i)];
            mx = nmax(mx, partial[2 * ((size_t)b * nper + i) + 1]);
        }
        const double bs = block_sum<kRedThreads>(s, red);
        const double bm = block_max<kRedThreads>(mx, red);
        if (threadIdx.x == 0) {
            mu[b] = bs / npts;
            gmax = nmax(gmax, bm);
        }
    }
    if (threadIdx.x == 0 && maxf) *maxf = gmax;
}

hipError_t launch_finalize_xfwd(const double* partial, int nper, int batch, double npts, double* mu, double* maxf,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_xfwd, dim3(1), dim3(kRedThreads), 0, s, partial, nper, batch, npts, mu, maxf);
    return hipGetLastError();
}

// Refinement bookkeeping after an update: gauge shift per batch entry (mean of
// u over the gauge region, removed by the next update), the size of the last
// correction relative to u, and the power-of-two scale of the next residual so
// that its float image stays well inside the float range.
__global__ __launch_bounds__(kRedThreads) void k_finalize_update(const double* __restrict__ partial, int nper,
                                                                 int batch, double nregion,
                                                                 double* __restrict__ sc, int first) {
    __shared__ double red[kRedThreads / 64];
    double gd = 0.0, gu = 0.0;
    for (int b = 0; b < batch; ++b) {
        double s = 0.0, md = 0.0, mu = 0.0;
        for (int i = threadIdx.x; i < nper; i += kRedThreads) {
            const size_t k = 3 * ((size_t)b * nper + i);
            s += partial[k];
            md = nmax(md, partial[k + 1]);
            mu = nmax(mu, partial[k + 2]);
        }
        const double bs = block_sum<kRedThreads>(s, red);
        const double bd = block_max<kRedThreads>(md, red);
        const double bu = block_max<kRedThreads>(mu, red);
        if (threadIdx.x == 0) {
            sc[SC_COUNT + 2 * batch + b] = nregion > 0.0 ? bs / nregion : 0.0;
            gd = nmax(gd, bd);
            gu = nmax(gu, bu);
        }
    }
    if (threadIdx.x == 0) {
        const double rel = (gu == 0.0) ? 0.0 : gd / gu;   // NaN stays NaN
        sc[SC_RELPREV] = first ? 1.0 : sc[SC_REL];
        sc[SC_MAXD] = gd;
        sc[SC_MAXU] = gu;
        sc[SC_REL] = rel;
        const double est = sc[SC_MAXF] * (rel > 0.0 ? rel : 1.0);
        int e = 0;
        if (est > 0.0 && isfinite(est)) e = ilogb(est);
        e = max(-1000, min(1000, e));
        sc[SC_SCALE] = ldexp(1.0, -e);
        sc[SC_INVSCALE] = ldexp(1.0, e);
    }
}

hipError_t launch_finalize_update(const double* partial, int nper, int batch, double nregion, double* scalars,
                                  int first, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_update, dim3(1), dim3(kRedThreads), 0, s, partial, nper, batch, nregion, scalars,
                       first);
    return hipGetLastError();
}

// r = scale * (f - lift - c - L_h u) in double, stored as float (lift: the face
// values of a non-homogeneous problem, see FaceArgs; c: see ResidualArgs;
// removing it in double keeps the float image of r at the precision of the
// small correction it carries).  L_h: the 7-point stencil of Eq. 3 with the
// face ghost rules (periodic wrap; Dirichlet ghost = -u of the boundary cell,
// linear extrapolation to a zero face value; Neumann ghost = u of the boundary
// cell).
//
// Every neighbour is read from a valid address: past a face the thread reads
// the periodic image, or the boundary cell itself and multiplies it by -1
// (Dirichlet) or +1 (Neumann).  The loads then carry no branches, and the
// values of the next plane are fetched while the current one is formed.
struct Nbr {
    long off;     // element offset of the value to read
    double sgn;   // factor applied to it
};

__device__ __forceinline__ Nbr neighbour(int idx, int n, long stride, int dir, int kind) {
    const int q = idx + dir;
    if (q >= 0 && q < n) return {(long)dir * stride, 1.0};
    if (kind == BC_P) return {(long)(dir < 0 ? (n - 1) : -(n - 1)) * stride, 1.0};
    return {0, kind == BC_D ? -1.0 : 1.0};
}

// One thread per (x, y) column and a stretch of kResZ planes: the z neighbours
// come from a three-plane window in registers, the x and y neighbours from the
// caches (their lines are loaded by the neighbouring threads of the block).
constexpr int kResZ = 16;

struct ResPlane {
    double xm, xp, ym, yp;   // in-plane neighbours (ghost rule applied)
    double up;               // the cell above (plane k + 1, ghost rule applied)
    double f;                // source
};

// Tu: the solution's type (float for the first solve of the refinement, double
// after); Tr: the residual's (double where its float rounding would limit the
// next correction, see the plan code).
template <typename Tu, typename Tr>
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ f, const Tu* __restrict__ u,
                                                  Tr* __restrict__ r, ResidualArgs a,
                                                  const double* __restrict__ sc) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    const int nzc = (a.nz + kResZ - 1) / kResZ;
    const int b = blockIdx.z / nzc;
    const int z0 = (blockIdx.z - b * nzc) * kResZ;
    if (i >= a.nx || j >= a.ny) return;
    const int z1 = min(z0 + kResZ, a.nz);
    const long plane = (long)a.nx * a.ny;
    const size_t base = (size_t)b * a.nz * plane + (size_t)j * a.nx + i;
    const Tu* ub = u + base;
    const double* fb = f + base;
    const double mu = a.proj ? sc[SC_COUNT + 3 * a.batch + b] : 0.0;
    const double scale = sc[SC_SCALE];
    const Nbr xm = neighbour(i, a.nx, 1, -1, a.bc[0]), xp = neighbour(i, a.nx, 1, 1, a.bc[1]);
    const Nbr ym = neighbour(j, a.ny, a.nx, -1, a.bc[2]), yp = neighbour(j, a.ny, a.nx, 1, a.bc[3]);
    auto load = [&](int k) {
        const Tu* p = ub + (long)k * plane;
        const Nbr zp = neighbour(k, a.nz, plane, 1, a.bc[5]);
        ResPlane v;
        v.xm = xm.sgn * (double)p[xm.off];
        v.xp = xp.sgn * (double)p[xp.off];
        v.ym = ym.sgn * (double)p[ym.off];
        v.yp = yp.sgn * (double)p[yp.off];
        v.up = zp.sgn * (double)p[zp.off];
        v.f = ld_stream(fb + (long)k * plane);
        return v;
    };
    // window: below, centre
    double uc = (double)ub[(long)z0 * plane];
    const Nbr zm = neighbour(z0, a.nz, plane, -1, a.bc[4]);
    double ud = zm.sgn * (double)ub[(long)z0 * plane + zm.off];
    ResPlane cur = load(z0);
    for (int k = z0; k < z1; ++k) {
        const ResPlane nxt = load(min(k + 1, z1 - 1));   // the last pass re-reads its own plane
        // second differences as sums of first differences: neighbouring values
        // of a smooth u differ by far less than their size, so each first
        // difference is exact (Sterbenz) and the stencil's rounding error scales
        // with |L_h u| rather than with |u| / h^2
        const double lx = (cur.xm - uc) + (cur.xp - uc);
        const double ly = (cur.ym - uc) + (cur.yp - uc);
        const double lz = (ud - uc) + (cur.up - uc);
        const double lap = lx * a.ihx2 + ly * a.ihy2 + lz * a.ihz2;
        double fi = cur.f;
        if (a.has_faces) fi -= face_lift(a.faces, b, i, j, k, a.nx, a.ny, a.nz);
        if (a.proj == 1) fi -= mu;
        else if (a.proj == 2 && k == 0) fi -= (double)a.nz * mu;
        st_stream(r + base + (size_t)k * plane, (Tr)((fi - lap) * scale));
        ud = uc;
        uc = cur.up;
        cur = nxt;
    }
}

template <typename Tu, typename Tr>
hipError_t launch_residual(const double* f, const Tu* u, Tr* r, const ResidualArgs& a, const double* scalars,
                           hipStream_t s) {
    const int nzc = (a.nz + kResZ - 1) / kResZ;
    dim3 grid((a.nx + 63) / 64, (a.ny + 3) / 4, nzc * a.batch);
    hipLaunchKernelGGL((k_residual<Tu, Tr>), grid, dim3(64, 4), 0, s, f, u, r, a, scalars);
    return hipGetLastError();
}
template hipError_t launch_residual<float, double>(const double*, const float*, double*, const ResidualArgs&,
                                                   const double*, hipStream_t);
template hipError_t launch_residual<double, double>(const double*, const double*, double*, const ResidualArgs&,
                                                    const double*, hipStream_t);
template hipError_t launch_residual<double, float>(const double*, const double*, float*, const ResidualArgs&,
                                                   const double*, hipStream_t);

// Streaming copy of n16 16-byte chunks: the bandwidth reference the solver's
// kernels are measured against (every kernel of the solve streams its input once
// and its output once).  Each workgroup moves contiguous tiles of 256 x
// kCopyUnroll chunks, all loads of a tile issued before its stores, with
// non-temporal loads and stores; 32 workgroups per CU.  (Measured on 1 GiB:
// 5.66 TB/s, against 4.3-5.0 TB/s for grid-stride forms and 5.2 TB/s for
// torch's copy.)
constexpr int kCopyUnroll = 8;
__global__ __launch_bounds__(256) void k_stream_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                     size_t n16) {
    constexpr size_t tile = 256 * kCopyUnroll;
    const size_t ntiles = n16 / tile;
    for (size_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const size_t base = t * tile + threadIdx.x;
        double2 v[kCopyUnroll];
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) v[k] = ld_stream(src + base + k * 256);
#pragma unroll
        for (int k = 0; k < kCopyUnroll; ++k) st_stream(dst + base + k * 256, v[k]);
    }
    // the tail after the last whole tile
    for (size_t i = ntiles * tile + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * blockDim.x)
        st_stream(dst + i, ld_stream(src + i));
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const int cus = device_cus();
    hipLaunchKernelGGL(k_stream_copy, dim3(cus * 32), dim3(256), 0, s, reinterpret_cast<const double2*>(src),
                       reinterpret_cast<double2*>(dst), bytes / 16);
    return hipGetLastError();
}

// Set the scalars that the first (unrefined) float solve reads in update mode.
__global__ void k_ir_init(double* sc, int batch) {
    const int t = threadIdx.x;
    if (t == 0) {
        sc[SC_SCALE] = 1.0;
        sc[SC_INVSCALE] = 1.0;
        sc[SC_REL] = 1.0;
        sc[SC_RELPREV] = 1.0;
    }
    for (int b = t; b < batch; b += blockDim.x) sc[SC_COUNT + 2 * batch + b] = 0.0;
}

hipError_t launch_ir_init(double* scalars, int batch, hipStream_t s) {
    hipLaunchKernelGGL(k_ir_init, dim3(1), dim3(64), 0, s, scalars, batch);
    return hipGetLastError();
}

}  // namespace pp
