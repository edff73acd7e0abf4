// The z-march: y transforms fused with the tridiagonal solves along z.
//
// One workgroup owns one spectral x column (slot m) of one batch entry: the
// ny x nz block S[b][m][:, :].  It marches z upward in chunks of zb planes:
//   load chunk -> forward y transform of every plane (LDS FFT + post-process)
//   -> forward elimination of the Thomas algorithm for every (entry, part)
//   -> store the eliminated right-hand sides in place;
// then downward:
//   load chunk -> back substitution -> inverse y transform -> store.
// The z-systems are those of section "Solution of the Resulting Tridiagonal
// Matrices": after the two transforms each (kx, ky) pair gives
//     (u_{k-1} - 2 u_k + u_{k+1}) / hz^2 + (lam_x + lam_y) u_k = fhat_k
// with lam from Table eig, a Toeplitz system whose boundary conditions only
// touch the first and last rows (Algorithm Thomas for Toeplitz Matrices).
// Multiplied by hz^2 its off-diagonals are 1, so elimination needs only the
// reciprocal pivots w_k = 1 / (b_k - w_{k-1}):
//     forward:  d'_k = (d_k - d'_{k-1}) w_k        back:  u_k = d'_k - w_k u_{k+1}
// The w_k depend on the wavenumbers only; the host tabulates them per line up
// to the index where they become constant in floating point (w_inf), plus the
// last row.  The singular zero mode is pinned by w_0 = 0 (its first unknown is
// held at zero, section "Well-posedness").
//
// y transforms (Table TransformationList, y faces): periodic -> complex DFT;
// Neumann -> DCT-II; Dirichlet -> DST-II stored reversed (entry e = DST index
// ny-1-e).  They act on complex lines linearly, so the two real x spectra of
// a DCT/DST slot (real and imaginary parts) are transformed together.  A
// periodic y transform of such a slot mixes the two parts; the pair
// (k, ny-k) is then separated into the two spectra
//     A_k = (Z_k + conj Z_{ny-k}) / 2 -> entry k,  B_k = (Z_k - conj Z_{ny-k}) / (2i) -> entry ny-k
// so that every entry's real and imaginary parts are independent z-systems.

#include "pp_kernels.hpp"

namespace pp {

// Reciprocal pivot of row z for an owned entry: the last row, a tabulated row
// (z < lmax), or the converged value.
template <typename T>
__device__ __forceinline__ cplx<T> pivot(const MidArgs<T>& a, int lmax, int roff, int z, int e, cplx<T> winf,
                                         cplx<T> wlast) {
    if (z == a.nz - 1) return wlast;
    if (z < lmax) return a.wrows[(size_t)(roff + z) * a.ny + e];
    return winf;
}

// Planes whose pivots and right-hand sides are fetched ahead of each stretch of
// the (serial) forward recurrence.
constexpr int kZBatch = 4;

// Global -> registers: this thread's entries e = tid + q*NTH (q < OWN) of the
// nl planes starting at z0, register l*OWN + q.  nl * OWN <= EPT.
template <typename T, int NTH, int EPT, int OWN>
__device__ __forceinline__ void fetch_owned(cplx<T> (&r)[EPT], const cplx<T>* __restrict__ col, int z0, int nl,
                                            int ny) {
#pragma unroll
    for (int l = 0; l < EPT / OWN; ++l) {
#pragma unroll
        for (int q = 0; q < OWN; ++q) {
            const int e = threadIdx.x + q * NTH;
            if (l < nl && e < ny) r[l * OWN + q] = col[(size_t)(z0 + l) * ny + e];
        }
    }
}

template <typename T, int NTH, int EPT, int OWN>
__global__ __launch_bounds__(NTH) void k_zmarch(cplx<T>* __restrict__ S, MidArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    const int m = blockIdx.x, b = blockIdx.y;
    const int ny = a.ny, nz = a.nz, ldy = a.ldy, zb = a.zb;
    const int tid = threadIdx.x;
    cplx<T>* col = S + ((size_t)b * a.slots + m) * (size_t)nz * ny;
    const bool pairslot = (a.bx != BC_P) || (m == 0);
    const bool sep = (a.by == BC_P) && pairslot;
    const bool sing = a.singular && (m == 0);
    const int lmax = a.lmax[m], roff = a.rowoff[m];
    const T scale = a.scale;
    const T proj = (sing && a.project) ? (T)(a.hz2 * a.mu[b]) : T(0);
    const int half = (ny >> 1) + 1;
    const int nchunks = (nz + zb - 1) / zb;
    const float inv_ny = 1.0f / (float)ny, inv_half = 1.0f / (float)half;

    // owned entries: e = tid + q * NTH; converged and last-row pivots kept in registers
    cplx<T> st[OWN], winf[OWN], wlast[OWN];
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
        const int e = tid + q * NTH;
        st[q] = mk<T>(T(0), T(0));
        winf[q] = st[q];
        wlast[q] = st[q];
        if (e < ny) {
            winf[q] = a.winf[(size_t)m * ny + e];
            wlast[q] = a.wlast[(size_t)m * ny + e];
        }
    }

    cplx<T> pre[EPT];
    // ------------------------------------------------------------- upward
    fetch_owned<T, NTH, EPT, OWN>(pre, col, 0, min(zb, nz), ny);
    for (int c = 0; c < nchunks; ++c) {
        const int zc = c * zb;
        const int nl = min(zb, nz - zc);
        // prefetched values -> LDS, pre-processed for the y transform
#pragma unroll
        for (int l = 0; l < EPT / OWN; ++l) {
#pragma unroll
            for (int q = 0; q < OWN; ++q) {
                const int y = tid + q * NTH;
                if (l < nl && y < ny) {
                    cplx<T> v = pre[l * OWN + q];
                    int pos = y;
                    if (a.by != BC_P) {
                        pos = makhoul_pos(y, ny);
                        if (a.by == BC_D && (y & 1)) v = mk<T>(-v.x, -v.y);
                    }
                    lds[l * ldy + pad(pos)] = v;
                }
            }
        }
        if (c + 1 < nchunks) fetch_owned<T, NTH, EPT, OWN>(pre, col, zc + zb, min(zb, nz - zc - zb), ny);
        __syncthreads();
        fft_lines<NTH, EPT, false, T>(lds, ldy, nl, a.fy, a.twy);
        if (a.by != BC_P) {
            // DCT-II post-twiddle over the pairs (k, ny-k)
            for (int i = tid; i < nl * half; i += NTH) {
                const int l = fdiv(i, inv_half), k = i - l * half;
                if (k == 0) continue;
                cplx<T>* line = lds + l * ldy;
                const cplx<T> vk = line[pad(k)];
                const cplx<T> wk = a.mky[k];
                if (2 * k == ny) {
                    const cplx<T> cc = cadd(cmul(wk, vk), cmulc(vk, wk));
                    line[pad(k)] = cscale(cc, T(0.5));
                } else {
                    const cplx<T> vr = line[pad(ny - k)];
                    const cplx<T> wr = a.mky[ny - k];
                    line[pad(k)] = cscale(cadd(cmul(wk, vk), cmulc(vr, wk)), T(0.5));
                    line[pad(ny - k)] = cscale(cadd(cmul(wr, vr), cmulc(vk, wr)), T(0.5));
                }
            }
            __syncthreads();
        } else if (sep) {
            for (int i = tid; i < nl * half; i += NTH) {
                const int l = fdiv(i, inv_half), k = i - l * half;
                if (k == 0 || 2 * k >= ny) continue;
                cplx<T>* line = lds + l * ldy;
                const cplx<T> zk = line[pad(k)], zr = line[pad(ny - k)];
                line[pad(k)] = mk<T>(T(0.5) * (zk.x + zr.x), T(0.5) * (zk.y - zr.y));
                line[pad(ny - k)] = mk<T>(T(0.5) * (zk.y + zr.y), T(0.5) * (zr.x - zk.x));
            }
            __syncthreads();
        }
        // forward elimination, kZBatch planes at a time (pivots fetched before the
        // recurrence); the eliminated right-hand sides go straight back to HBM
#pragma unroll
        for (int q = 0; q < OWN; ++q) {
            const int e = tid + q * NTH;
            if (e < ny) {
                cplx<T> prev = st[q];
                for (int l0 = 0; l0 < nl; l0 += kZBatch) {
                    cplx<T> w[kZBatch], d[kZBatch];
#pragma unroll
                    for (int j = 0; j < kZBatch; ++j) {
                        const int l = l0 + j;
                        if (l < nl) {
                            w[j] = pivot(a, lmax, roff, zc + l, e, winf[q], wlast[q]);
                            d[j] = cscale(lds[l * ldy + pad(e)], scale);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < kZBatch; ++j) {
                        const int l = l0 + j;
                        if (l < nl) {
                            cplx<T> dd = d[j];
                            if (sing && e == 0) dd.x -= proj;
                            prev = mk<T>((dd.x - prev.x) * w[j].x, (dd.y - prev.y) * w[j].y);
                            col[(size_t)(zc + l) * ny + e] = prev;
                        }
                    }
                }
                st[q] = prev;
            }
        }
        __syncthreads();
    }

    // ----------------------------------------------------------- downward
    // Each thread's eliminated values come back in its own prefetch registers,
    // so back substitution runs on registers and only the result goes to LDS.
#pragma unroll
    for (int q = 0; q < OWN; ++q) st[q] = mk<T>(T(0), T(0));
    double csum = 0.0;
    {
        const int zc = (nchunks - 1) * zb;
        fetch_owned<T, NTH, EPT, OWN>(pre, col, zc, nz - zc, ny);
    }
    for (int c = nchunks - 1; c >= 0; --c) {
        const int zc = c * zb;
        const int nl = min(zb, nz - zc);
#pragma unroll
        for (int q = 0; q < OWN; ++q) {
            const int e = tid + q * NTH;
            if (e < ny) {
                cplx<T> nxt = st[q];
#pragma unroll
                for (int l = EPT / OWN - 1; l >= 0; --l) {
                    if (l < nl) {
                        const cplx<T> w = pivot(a, lmax, roff, zc + l, e, winf[q], wlast[q]);
                        const cplx<T> dp = pre[l * OWN + q];
                        nxt = mk<T>(dp.x - w.x * nxt.x, dp.y - w.y * nxt.y);
                        lds[l * ldy + pad(e)] = nxt;
                        if (sing && e == 0) csum += (double)nxt.x;
                    }
                }
                st[q] = nxt;
            }
        }
        if (c > 0) fetch_owned<T, NTH, EPT, OWN>(pre, col, zc - zb, zb, ny);
        __syncthreads();
        if (a.by != BC_P) {
            // DCT-III pre-twiddle: W_k = e^{+i pi k/2N} (X_k - i X_{N-k}), X_N = 0
            for (int i = tid; i < nl * half; i += NTH) {
                const int l = fdiv(i, inv_half), k = i - l * half;
                if (k == 0) continue;
                cplx<T>* line = lds + l * ldy;
                const cplx<T> xk = line[pad(k)];
                if (2 * k == ny) {
                    line[pad(k)] = cmulc(mk<T>(xk.x + xk.y, xk.y - xk.x), a.mky[k]);
                } else {
                    const cplx<T> xr = line[pad(ny - k)];
                    line[pad(k)] = cmulc(mk<T>(xk.x + xr.y, xk.y - xr.x), a.mky[k]);
                    line[pad(ny - k)] = cmulc(mk<T>(xr.x + xk.y, xr.y - xk.x), a.mky[ny - k]);
                }
            }
            __syncthreads();
        } else if (sep) {
            for (int i = tid; i < nl * half; i += NTH) {
                const int l = fdiv(i, inv_half), k = i - l * half;
                if (k == 0 || 2 * k >= ny) continue;
                cplx<T>* line = lds + l * ldy;
                const cplx<T> A = line[pad(k)], B = line[pad(ny - k)];
                line[pad(k)] = mk<T>(A.x - B.y, A.y + B.x);        // A + i B
                line[pad(ny - k)] = mk<T>(A.x + B.y, B.x - A.y);   // conj(A) + i conj(B)
            }
            __syncthreads();
        }
        fft_lines<NTH, EPT, true, T>(lds, ldy, nl, a.fy, a.twy);
        for (int i = tid; i < nl * ny; i += NTH) {
            const int l = fdiv(i, inv_ny), y = i - l * ny;
            int pos = y;
            if (a.by != BC_P) pos = makhoul_pos(y, ny);
            cplx<T> v = lds[l * ldy + pad(pos)];
            if (a.by == BC_D && (y & 1)) v = mk<T>(-v.x, -v.y);
            col[(size_t)(zc + l) * ny + y] = v;
        }
        __syncthreads();
    }
    if (m == 0 && tid == 0) a.cmean[b] = (sing && a.demean) ? csum / (double)nz : 0.0;
}

template <typename T, int OWN>
static hipError_t launch_mid_own(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s) {
    const size_t lds = (size_t)a.zb * a.ldy * sizeof(cplx<T>);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_zmarch<T, kZThreads, kEpt, OWN>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)((kZElems + kZElems / 8) * sizeof(cplx<double>)));
        attr = true;
    }
    hipLaunchKernelGGL((k_zmarch<T, kZThreads, kEpt, OWN>), dim3(a.slots, batch), dim3(kZThreads), lds, s, S, a);
    return hipGetLastError();
}

// Entries per thread: ceil(ny / kZThreads) <= kZOwned.
template <typename T>
hipError_t launch_mid(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s) {
    const int own = (a.ny + kZThreads - 1) / kZThreads;
    if (own <= 1) return launch_mid_own<T, 1>(S, a, batch, s);
    if (own <= 2) return launch_mid_own<T, 2>(S, a, batch, s);
    return launch_mid_own<T, kZOwned>(S, a, batch, s);
}

template hipError_t launch_mid<double>(cplx<double>*, const MidArgs<double>&, int, hipStream_t);
template hipError_t launch_mid<float>(cplx<float>*, const MidArgs<float>&, int, hipStream_t);

}  // namespace pp
