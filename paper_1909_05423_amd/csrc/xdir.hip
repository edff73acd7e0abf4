// x-direction kernels: forward real transform of every x row with the
// transpose into the spectral layout, and the inverse transform back to rows.
//
// Forward (Table TransformationList, x faces):
//   periodic  -> DFT of the real row (Eq. for the periodic condition),
//   Neumann   -> DCT-II (Neumann subsection),
//   Dirichlet -> DST-II (Dirichlet subsection), computed as the DCT-II of
//                (-1)^n u_n read in reverse order: DST-II(u)_k = DCT-II((-1)^n u)_{N-1-k}.
// Two real rows share one complex line (row 2j in the real part, row 2j+1 in
// the imaginary part), so one complex FFT serves two rows.  The DCT-II uses
// the reordering of the Neumann subsection (even samples ascending, odd
// samples descending) and the post-twiddle pairing k with N-k, which is the
// "Hermitian symmetry" step written so it stays linear over complex lines:
//     C_k = 1/2 (e^{-i pi k/2N} V_k + e^{+i pi k/2N} V_{N-k}),  V_N = V_0.
// The Dirichlet output is stored unreversed: spectral column k holds DST
// index N-1-k (the z-solve tables carry that mapping).
//
// Spectral layout S[b][m][z][y] (complex): y contiguous, m = spectral column
// slot, ceil(nx/2) slots per row:
//   periodic x:  slot 0 = (X_0, X_{nx/2}) (both real; X_{nx/2} = 0 for odd nx),
//                slot m = X_m for 1 <= m < ceil(nx/2);
//   DCT / DST :  slot m = (C_{2m}, C_{2m+1})  (C_{nx} = 0 for odd nx).
// Writing columns with y contiguous is the x <-> y transpose, done through LDS
// so that both the row reads and the column writes are coalesced.

#include "pp_kernels.hpp"

namespace pp {

// One DCT-II bin of a packed pair of rows, from the DFT V of the reordered
// complex line: C_k = 1/2 (e^{-i pi k/2N} V_k + e^{+i pi k/2N} V_{N-k}), V_N = V_0.
template <typename T>
__device__ __forceinline__ cplx<T> dct_bin(const cplx<T>* line, const cplx<T>* __restrict__ mkt, int k, int N) {
    const cplx<T> vk = line[pad(k)];
    const cplx<T> vr = line[pad(k == 0 ? 0 : N - k)];
    const cplx<T> w = mkt[k];
    return cscale(cadd(cmul(w, vk), cmulc(vr, w)), T(0.5));
}

template <typename T, typename Tin, int NTH>
__global__ __launch_bounds__(NTH) void k_xfwd(const Tin* __restrict__ f, cplx<T>* __restrict__ S,
                                              double* __restrict__ partial, XArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    __shared__ double red[NTH / 64];
    const int nx = a.nx, ny = a.ny, nz = a.nz, ty = a.ty, ldl = a.ldl;
    const int y0 = blockIdx.x * ty, z = blockIdx.y, b = blockIdx.z;
    const int tid = threadIdx.x;
    const Tin* src = f + ((size_t)b * nz + z) * (size_t)ny * nx;

    // 1. rows -> packed complex lines (row 2j real part, row 2j+1 imaginary part),
    //    pre-processed for the x transform
    double acc = 0.0, amax = 0.0;
    const int nlines = ty >> 1;
    const float inv_nx = 1.0f / (float)nx, inv_nl = 1.0f / (float)nlines;
    for (int i = tid; i < nlines * nx; i += NTH) {
        const int j = fdiv(i, inv_nx), n = i - j * nx;
        const int ya = y0 + 2 * j, yb = ya + 1;
        T va = T(0), vb = T(0);
        if (ya < ny) {
            const Tin raw = src[(size_t)ya * nx + n];
            acc += (double)raw;
            amax = fmax(amax, fabs((double)raw));
            va = (T)raw;
        }
        if (yb < ny) {
            const Tin raw = src[(size_t)yb * nx + n];
            acc += (double)raw;
            amax = fmax(amax, fabs((double)raw));
            vb = (T)raw;
        }
        int pos = n;
        if (a.bx != BC_P) {
            pos = makhoul_pos(n, nx);
            if (a.bx == BC_D && (n & 1)) {
                va = -va;
                vb = -vb;
            }
        }
        lds[j * ldl + pad(pos)] = mk<T>(va, vb);
    }
    const double bsum = block_sum<NTH>(acc, red);
    const double bmax = block_max<NTH>(amax, red);
    if (tid == 0) {
        const size_t blk = ((size_t)b * gridDim.y + z) * gridDim.x + blockIdx.x;
        partial[2 * blk] = bsum;
        partial[2 * blk + 1] = bmax;
    }
    __syncthreads();

    // 2. complex FFT of every line
    fft_lines<NTH, kEpt, false, T>(lds, ldl, ty >> 1, a.fx, a.twx);

    // 3. post-process and write columns (y contiguous); one thread per (slot, row pair)
    cplx<T>* dstS = S + (size_t)b * a.slots * nz * ny;
    for (int i = tid; i < a.slots * nlines; i += NTH) {
        const int m = fdiv(i, inv_nl), j = i - m * nlines;
        const int ya = y0 + 2 * j, yb = ya + 1;
        const cplx<T>* line = lds + j * ldl;
        cplx<T> oa, ob;
        if (a.bx == BC_P) {
            if (m == 0) {
                const cplx<T> z0 = line[pad(0)];
                // X_a[0] = Re Z_0, X_b[0] = Im Z_0; likewise at the Nyquist bin
                cplx<T> zn = mk<T>(T(0), T(0));
                if (!(nx & 1)) zn = line[pad(nx >> 1)];
                oa = mk<T>(z0.x, zn.x);
                ob = mk<T>(z0.y, zn.y);
            } else {
                // X_a[m] = (Z_m + conj Z_{N-m}) / 2,  X_b[m] = (Z_m - conj Z_{N-m}) / (2i)
                const cplx<T> zk = line[pad(m)], zr = line[pad(nx - m)];
                oa = mk<T>(T(0.5) * (zk.x + zr.x), T(0.5) * (zk.y - zr.y));
                ob = mk<T>(T(0.5) * (zk.y + zr.y), T(0.5) * (zr.x - zk.x));
            }
        } else {
            // C_k = 1/2 (e^{-i pi k/2N} V_k + e^{+i pi k/2N} V_{N-k}); real part -> row a, imaginary -> row b
            const int k0 = 2 * m, k1 = 2 * m + 1;
            const cplx<T> c0 = dct_bin<T>(line, a.mkx, k0, nx);
            const cplx<T> c1 = (k1 < nx) ? dct_bin<T>(line, a.mkx, k1, nx) : mk<T>(T(0), T(0));
            oa = mk<T>(c0.x, c1.x);
            ob = mk<T>(c0.y, c1.y);
        }
        const size_t col = ((size_t)m * nz + z) * ny;
        if (ya < ny) dstS[col + ya] = oa;
        if (yb < ny) dstS[col + yb] = ob;
    }
}

// Inverse x transform of one z plane slab: spectral columns -> rows.
//   periodic  -> complex-to-real inverse DFT, unnormalised (returns N x);
//   DCT / DST -> 2 * DCT-III by the inverse of the reordering scheme
//                (Neumann subsection): W_k = e^{+i pi k/2N} (X_k - i X_{N-k}),
//                X_N = 0, v = IDFT_unnormalised(W), x_{2m} = v_m,
//                x_{2m+1} = v_{N-1-m}; Dirichlet multiplies x_n by (-1)^n
//                (its spectral columns are already stored reversed).
// MODE XINV_STORE writes u = x - shift[b]; XINV_UPDATE adds to a double u.
template <typename T, typename Tout, int NTH, int MODE>
__global__ __launch_bounds__(NTH) void k_xinv(const cplx<T>* __restrict__ S, Tout* __restrict__ u, XArgs<T> a,
                                              const double* __restrict__ shift, const double* __restrict__ scalars,
                                              int gauge_region, double* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    __shared__ double red[NTH / 64];
    const int nx = a.nx, ny = a.ny, nz = a.nz, ty = a.ty, ldl = a.ldl;
    const int y0 = blockIdx.x * ty, z = blockIdx.y, b = blockIdx.z;
    const int tid = threadIdx.x;
    const int nlines = ty >> 1;
    const cplx<T>* srcS = S + (size_t)b * a.slots * nz * ny;
    const float inv_nl = 1.0f / (float)nlines, inv_nx = 1.0f / (float)nx;

    // 1. columns -> packed complex spectra of row pairs
    for (int i = tid; i < a.slots * nlines; i += NTH) {
        const int m = fdiv(i, inv_nl), j = i - m * nlines;
        const int ya = y0 + 2 * j, yb = ya + 1;
        const size_t col = ((size_t)m * nz + z) * ny;
        const cplx<T> sa = (ya < ny) ? srcS[col + ya] : mk<T>(T(0), T(0));
        const cplx<T> sb = (yb < ny) ? srcS[col + yb] : mk<T>(T(0), T(0));
        cplx<T>* line = lds + j * ldl;
        if (a.bx == BC_P) {
            if (m == 0) {
                line[pad(0)] = mk<T>(sa.x, sb.x);
                if (!(nx & 1)) line[pad(nx >> 1)] = mk<T>(sa.y, sb.y);
            } else {
                line[pad(m)] = mk<T>(sa.x - sb.y, sa.y + sb.x);        // X_a + i X_b
                line[pad(nx - m)] = mk<T>(sa.x + sb.y, sb.x - sa.y);   // conj(X_a) + i conj(X_b)
            }
        } else {
            line[pad(2 * m)] = mk<T>(sa.x, sb.x);
            if (2 * m + 1 < nx) line[pad(2 * m + 1)] = mk<T>(sa.y, sb.y);
        }
    }
    __syncthreads();
    if (a.bx != BC_P) {
        const int half = (nx >> 1) + 1;
        const float inv_half = 1.0f / (float)half;
        for (int i = tid; i < nlines * half; i += NTH) {
            const int j = fdiv(i, inv_half), k = i - j * half;
            if (k == 0) continue;                       // W_0 = X_0
            cplx<T>* line = lds + j * ldl;
            const cplx<T> xk = line[pad(k)];
            if (2 * k == nx) {
                line[pad(k)] = cmulc(mk<T>(xk.x + xk.y, xk.y - xk.x), a.mkx[k]);   // e^{+} (X_k - i X_k)
            } else {
                const cplx<T> xr = line[pad(nx - k)];
                // X_k - i X_{N-k} = (xk.x + xr.y, xk.y - xr.x)
                line[pad(k)] = cmulc(mk<T>(xk.x + xr.y, xk.y - xr.x), a.mkx[k]);
                line[pad(nx - k)] = cmulc(mk<T>(xr.x + xk.y, xr.y - xk.x), a.mkx[nx - k]);
            }
        }
        __syncthreads();
    }

    // 2. inverse complex FFT (unnormalised)
    fft_lines<NTH, kEpt, true, T>(lds, ldl, nlines, a.fx, a.twx);

    // 3. rows out
    const double sh = shift ? shift[b] : 0.0;
    double inv_scale = 1.0, gshift = 0.0;
    if (MODE == XINV_UPDATE) {
        inv_scale = scalars[SC_INVSCALE];
        gshift = scalars[SC_COUNT + 2 * (int)gridDim.z + b];
    }
    double acc = 0.0, dmax = 0.0, umax = 0.0;
    Tout* dst = u + ((size_t)b * nz + z) * (size_t)ny * nx;
    for (int i = tid; i < nlines * nx; i += NTH) {
        const int j = fdiv(i, inv_nx), n = i - j * nx;
        int pos = n;
        if (a.bx != BC_P) pos = makhoul_pos(n, nx);
        cplx<T> c = lds[j * ldl + pad(pos)];
        if (a.bx == BC_D && (n & 1)) c = mk<T>(-c.x, -c.y);
#pragma unroll
        for (int part = 0; part < 2; ++part) {
            const int y = y0 + 2 * j + part;
            if (y >= ny) continue;
            const T v = part ? c.y : c.x;
            const size_t idx = (size_t)y * nx + n;
            if (MODE == XINV_STORE) {
                dst[idx] = (Tout)((double)v - sh);
            } else {
                const double d = ((double)v - sh) * inv_scale;
                const double un = (double)dst[idx] + d - gshift;
                dst[idx] = (Tout)un;
                if (gauge_region == 1 || (gauge_region == 2 && z == 0)) acc += un;
                dmax = fmax(dmax, fabs(d));
                umax = fmax(umax, fabs(un));
            }
        }
    }
    if (MODE == XINV_UPDATE) {
        const double bs = block_sum<NTH>(acc, red);
        const double bd = block_max<NTH>(dmax, red);
        const double bu = block_max<NTH>(umax, red);
        if (tid == 0) {
            const size_t blk = ((size_t)b * gridDim.y + z) * gridDim.x + blockIdx.x;
            partial[3 * blk] = bs;
            partial[3 * blk + 1] = bd;
            partial[3 * blk + 2] = bu;
        }
    }
}

template <typename T> static size_t x_lds_bytes(const XArgs<T>& a) {
    return (size_t)(a.ty >> 1) * a.ldl * sizeof(cplx<T>);
}

// Allow the kernel the full dynamic LDS budget (beyond the 64 KiB default).
template <typename K> static void allow_lds(K kernel) {
    static bool done = false;
    if (!done) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)((kXElems + kXElems / 8) * sizeof(cplx<double>)));
        done = true;
    }
}

template <typename T, typename Tin>
hipError_t launch_xfwd(const Tin* f, cplx<T>* S, double* partial, const XArgs<T>& a, int batch, hipStream_t s) {
    dim3 grid((a.ny + a.ty - 1) / a.ty, a.nz, batch);
    allow_lds(k_xfwd<T, Tin, kXThreads>);
    hipLaunchKernelGGL((k_xfwd<T, Tin, kXThreads>), grid, dim3(kXThreads), x_lds_bytes(a), s, f, S, partial, a);
    return hipGetLastError();
}

template <typename T, typename Tout>
hipError_t launch_xinv(const cplx<T>* S, Tout* u, const XArgs<T>& a, int batch, const double* shift, hipStream_t s) {
    dim3 grid((a.ny + a.ty - 1) / a.ty, a.nz, batch);
    allow_lds(k_xinv<T, Tout, kXThreads, XINV_STORE>);
    hipLaunchKernelGGL((k_xinv<T, Tout, kXThreads, XINV_STORE>), grid, dim3(kXThreads), x_lds_bytes(a), s, S, u, a,
                       shift, (const double*)nullptr, 0, (double*)nullptr);
    return hipGetLastError();
}

hipError_t launch_xinv_update(const cplx<float>* S, double* u, const XArgs<float>& a, int batch,
                              const double* scalars, int gauge_region, double* partial, hipStream_t s) {
    dim3 grid((a.ny + a.ty - 1) / a.ty, a.nz, batch);
    const double* shift = scalars + SC_COUNT + batch;   // cmean of the correction solve
    allow_lds(k_xinv<float, double, kXThreads, XINV_UPDATE>);
    hipLaunchKernelGGL((k_xinv<float, double, kXThreads, XINV_UPDATE>), grid, dim3(kXThreads), x_lds_bytes(a), s, S, u,
                       a, shift, scalars, gauge_region, partial);
    return hipGetLastError();
}

template hipError_t launch_xfwd<double, double>(const double*, cplx<double>*, double*, const XArgs<double>&, int,
                                                hipStream_t);
template hipError_t launch_xfwd<float, float>(const float*, cplx<float>*, double*, const XArgs<float>&, int,
                                              hipStream_t);
template hipError_t launch_xfwd<float, double>(const double*, cplx<float>*, double*, const XArgs<float>&, int,
                                               hipStream_t);
template hipError_t launch_xinv<double, double>(const cplx<double>*, double*, const XArgs<double>&, int,
                                                const double*, hipStream_t);
template hipError_t launch_xinv<float, float>(const cplx<float>*, float*, const XArgs<float>&, int, const double*,
                                              hipStream_t);
template hipError_t launch_xinv<float, double>(const cplx<float>*, double*, const XArgs<float>&, int,
                                               const double*, hipStream_t);

}  // namespace pp
