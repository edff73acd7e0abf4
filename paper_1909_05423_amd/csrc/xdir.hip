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

#include <mutex>
#include <set>
#include <tuple>
#include <type_traits>

#include "pp_kernels.hpp"

namespace pp {

// One DCT-II bin of a packed pair of rows, from the DFT V of the reordered
// complex line: C_k = 1/2 (e^{-i pi k/2N} V_k + e^{+i pi k/2N} V_{N-k}), V_N = V_0.
template <typename T>
__device__ __forceinline__ cplx<T> dct_bin(const cplx<T>* line, const cplx<T>* mkt, int k, int N) {
    const cplx<T> vk = line[pad(k)];
    const cplx<T> vr = line[pad(k == 0 ? 0 : N - k)];
    const cplx<T> w = mkt[k];
    return cscale(cadd(cmul(w, vk), cmulc(vr, w)), T(0.5));
}

// Block index -> (row block, z plane, batch entry) of the x kernels.
struct XBlock {
    int y0, z, b;
};
// Order in which a persistent x workgroup takes row blocks.  A block of 8 rows
// covers 8 consecutive entries of every spectral column: a whole 128-byte line
// with double spectra, half of one with float spectra.  The inverse kernel with
// float spectra (PAIR) therefore takes blocks in pairs 2p, 2p + 1 (the two
// halves of the same lines), one right after the other, so that the second
// finds the lines in its XCD's L2 instead of fetching them again; pairs follow
// at 2 gridDim.x.  Otherwise a workgroup takes blocks blockIdx.x + i gridDim.x.
// (Measured: pairing cut the float inverse's time by 6-11%; the forward
// kernel, whose float column writes are the halves, gained nothing from it.)
template <bool PAIR> __device__ __forceinline__ int x_first_block() {
    if constexpr (PAIR) return 2 * (int)blockIdx.x;
    else return (int)blockIdx.x;
}
template <bool PAIR> __device__ __forceinline__ int x_next_block(int blk) {
    if constexpr (PAIR) return (blk & 1) ? blk + 2 * (int)gridDim.x - 1 : blk + 1;
    else return blk + (int)gridDim.x;
}

// ends: z planes from both ends inward (XArgs::zends)
__device__ __forceinline__ XBlock x_block(int blk, int nyb, int nz, int ty, bool ends = false) {
    XBlock r;
    const int yb = blk % nyb;
    const int zz = blk / nyb;
    const int q = zz % nz;
    r.y0 = yb * ty;
    r.z = ends ? ((q & 1) ? nz - 1 - (q >> 1) : (q >> 1)) : q;
    r.b = zz / nz;
    return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nmax(v, __shfl_down(v, off, 64));
    return v;
}

// Store of one spectral value by the forward x kernel.  Float spectra are
// streamed past the caches; double spectra are stored normally (measured: the
// streaming store made the double solve slower and the float one faster).
template <typename T> __device__ __forceinline__ void put_spec(cplx<T>* p, const cplx<T>& v) {
    if constexpr (sizeof(T) == 4) st_stream(p, v);
    else *p = v;
}

// Forward x kernel, persistent: each workgroup walks row blocks in the order
// of x_first_block / x_next_block; the rows of the next block are in
// flight into registers while the current one is transformed.  Each wavefront
// transforms its own lines (line j = wave + NW p holds rows 2j, 2j+1; its lanes
// hold columns n = lane + 64 k) without workgroup barriers; the transposed
// write of the spectral columns reads across lines.  Partial sums of the source
// (sum, max |f|) are written per wavefront.
//
// Order of issue per block: lines from the prefetched rows, prefetch of the
// next block, transforms, column stores.  The wait for a prefetch then only
// has the previous block's stores behind it.  FULL (nx = 64 RMAX, one line per
// wavefront, ny a multiple of the block height) has no data-dependent branch
// around a memory instruction, so that count is exact; the first block is
// issued outside the loop so every pass through it sees the same sequence.
// Minimum waves per SIMD the compiler must leave room for.  2 for the
// all-float forward kernel on rows up to 512 and for the double kernel on
// rows of 512 without face values (4 registers over the budget of two waves);
// no constraint elsewhere: the kernels with double data, and the float kernel
// on rows of 1024, spill under it (the float one 104 registers, 3.0 ms at
// 1024 x 1024 x 512; unconstrained it takes AGPRs instead, one wave per SIMD,
// 1.75 ms).  The general form of the fused residual (RES) spills under it too.
template <typename T, typename Tin, int RMAX, bool FACES, bool FULL = true, bool RES = false>
constexpr int kXfwdMinWaves =
    (RES && !FULL) ? 1
                   : ((sizeof(T) == 4 && sizeof(Tin) == 4 && RMAX <= 8) || (sizeof(T) == 8 && RMAX == 8 && !FACES)) ? 2
                                                                                                                     : 1;

// RES: the fused refinement residual (XArgs::u0 ...): besides the source
// rows, each lane fetches its own u0 values of the two rows, of the rows
// outside the pair in y and of the neighbouring planes; the x neighbours come
// from the adjacent lanes (exact-count form) or from loads (general form).
// Neighbours past a face are read at a valid address (the periodic image, or
// the cell itself with the sign of the ghost rule) as in k_residual.
template <typename T, typename Tin, typename Ts, int NTH, int RMAX, bool FULL, bool FACES, bool RES = false>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(kXfwdMinWaves<T, Tin, RMAX, FACES, FULL, RES>))) void k_xfwd(const Tin* __restrict__ f, cplx<Ts>* __restrict__ S,
                                              double* __restrict__ partial, XArgs<T> a, int nblocks,
                                              FaceArgs<Tin> fa) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool SPLIT = !std::is_same_v<T, Ts>;   // double arithmetic, float spectra + double slots
    constexpr int NW = NTH / 64;
    constexpr int PAIRS = RMAX / 2;   // FULL: column writes per thread, slots * nlines == NTH * PAIRS
    const int nx = FULL ? 64 * RMAX : a.nx;
    const int ny = a.ny, nz = a.nz, ty = FULL ? 2 * NW : a.ty, ldl = a.ldl;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nlines = ty >> 1;
    const int nyb = (ny + ty - 1) / ty;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* twl = lds + nlines * ldl;
    cplx<T>* mkl = twl + nx;
    for (int i = tid; i < nx; i += NTH) {
        twl[i] = a.twx[i];
        mkl[i] = a.mkx[i];
    }
    const int epl = FULL ? RMAX : (nx + 63) >> 6;
    const float inv_epl = 1.0f / (float)epl, inv_nl = 1.0f / (float)nlines;
    // periodic rows of 512, double spectra: the transform's first stage runs
    // on the row registers (w512_first; in float the extra registers cost more
    // occupancy than the LDS round trip saves)
    // (not with the fused residual, whose neighbour values need the registers,
    // nor with the split store, which spilled with it)
    constexpr bool R512 = FULL && RMAX == 8 && sizeof(T) == 8 && !RES && !SPLIT;
    const bool reg512 = R512 && a.bx == BC_P;

    // register r: line j = wave + NW * (r / epl), column n = lane + 64 * (r % epl)
    Tin ra[RMAX], rb[RMAX];
    // RES: u0 at the two rows (ua, ub), at the row below a and above b (uya, uyb)
    // and at the planes below and above (uza0, uza1, uzb0, uzb1)
    constexpr int RR = RES ? RMAX : 1;
    float ua[RR], ub[RR], uya[RR], uyb[RR], uza0[RR], uza1[RR], uzb0[RR], uzb1[RR];
    // neighbour row / plane index past a face: the periodic image or the cell itself
    auto nb_idx = [&](int i, int n_, int dir, int kind) -> int {
        const int q = i + dir;
        if (q >= 0 && q < n_) return q;
        return kind == BC_P ? (q < 0 ? n_ - 1 : 0) : i;
    };
    auto nb_sgn = [&](int i, int n_, int dir, int kind) -> double {
        const int q = i + dir;
        return (q >= 0 && q < n_) || kind != BC_D ? 1.0 : -1.0;
    };
    // FULL with face values: the x-face values of this wave's two rows, fetched
    // with them (the lanes holding columns 0 and nx-1 use them)
    Tin gx[FACES && FULL ? 4 : 1];
    auto fetch = [&](int blk) {
        const XBlock xb = x_block(blk, nyb, nz, ty);
        if constexpr (FACES && FULL) {
            const size_t row = ((size_t)xb.b * nz + xb.z) * ny + xb.y0 + 2 * wave;
            gx[0] = fa.g[0][row];
            gx[1] = fa.g[0][row + 1];
            gx[2] = fa.g[1][row];
            gx[3] = fa.g[1][row + 1];
        }
        const Tin* src = f + ((size_t)xb.b * nz + xb.z) * (size_t)ny * nx;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int p = FULL ? 0 : fdiv(r, inv_epl);
            const int j = wave + NW * p, n = lane + 64 * (r - p * epl);
            const int ya = xb.y0 + 2 * j;
            if (FULL) {
                ra[r] = ld_stream(src + (size_t)ya * nx + n);
                rb[r] = ld_stream(src + (size_t)(ya + 1) * nx + n);
            } else {
                ra[r] = Tin(0);
                rb[r] = Tin(0);
                if (j < nlines && n < nx) {
                    if (ya < ny) ra[r] = ld_stream(src + (size_t)ya * nx + n);
                    if (ya + 1 < ny) rb[r] = ld_stream(src + (size_t)(ya + 1) * nx + n);
                }
            }
            if constexpr (RES) {
                // the pair's own u0 values travel with the source rows; the
                // neighbour rows are read when the block is formed (fetch_nb)
                const float* up = a.u0 + ((size_t)xb.b * nz + xb.z) * (size_t)ny * nx;
                const bool va = FULL || (j < nlines && n < nx && ya < ny);
                const bool vb = FULL || (j < nlines && n < nx && ya + 1 < ny);
                ua[r] = va ? up[(size_t)ya * nx + n] : 0.f;
                ub[r] = vb ? up[(size_t)(ya + 1) * nx + n] : 0.f;
            }
        }
    };
    // RES: u0 of the rows outside the pair in y (below a; above b, or above a
    // when b is past the end) and of the neighbouring planes, for block blk
    // (issued when the block is formed: issued one block ahead, after the
    // transform, they cost registers the kernel does not have, 3.00 -> 3.09 ms)
    auto fetch_nb = [&](int blk) {
        if constexpr (RES) {
            const XBlock xb = x_block(blk, nyb, nz, ty);
            const float* up = a.u0 + ((size_t)xb.b * nz + xb.z) * (size_t)ny * nx;
            const long plane = (long)ny * nx;
            const long zm = (long)(nb_idx(xb.z, nz, -1, a.fbc[4]) - xb.z) * plane;
            const long zp = (long)(nb_idx(xb.z, nz, 1, a.fbc[5]) - xb.z) * plane;
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                const int p = FULL ? 0 : fdiv(r, inv_epl);
                const int j = wave + NW * p, n = lane + 64 * (r - p * epl);
                const int ya = xb.y0 + 2 * j;
                const bool va = FULL || (j < nlines && n < nx && ya < ny);
                const bool vb = FULL || (j < nlines && n < nx && ya + 1 < ny);
                const int ym = nb_idx(ya, ny, -1, a.fbc[2]);
                const int yp = nb_idx(vb ? ya + 1 : ya, ny, 1, a.fbc[3]);
                const float* pa = up + (size_t)(va ? ya : 0) * nx + (va ? n : 0);
                const float* pb = up + (size_t)(vb ? ya + 1 : 0) * nx + (vb ? n : 0);
                uya[r] = va ? up[(size_t)ym * nx + n] : 0.f;
                uyb[r] = va ? up[(size_t)yp * nx + n] : 0.f;
                uza0[r] = va ? pa[zm] : 0.f;
                uza1[r] = va ? pa[zp] : 0.f;
                uzb0[r] = vb ? pb[zm] : 0.f;
                uzb1[r] = vb ? pb[zp] : 0.f;
            }
        }
    };
    // RES: the value of u0 at column n - 1 (dir -1) or n + 1 (dir +1) of the row
    // held in c (exact-count form: lane l holds columns l + 64 r), from the
    // adjacent lane; past the x faces the periodic image or the ghost rule
    // (DPP wave_ror:1 gives lane l the value of lane l - 1, lane 0 that of lane
    // 63; wave_rol:1 lane l + 1, lane 63 that of lane 0)
    auto rot1 = [&](float v, int dir) -> float {
        const int iv = __float_as_int(v);
        const int o = dir < 0 ? __builtin_amdgcn_update_dpp(0, iv, 0x13C, 0xF, 0xF, false)
                              : __builtin_amdgcn_update_dpp(0, iv, 0x134, 0xF, 0xF, false);
        return __int_as_float(o);
    };
    auto xnb = [&](const float (&c)[RR], int r, int dir) -> double {
        if constexpr (RES && FULL) {
            const int rw = (r + dir + RMAX) % RMAX;   // the register of the wrapped-around lane
            const float t1 = rot1(c[r], dir);
            const float t2 = rot1(c[rw], dir);
            const bool wrap = dir < 0 ? (lane == 0) : (lane == 63);
            const int n = lane + 64 * r;
            const bool face = dir < 0 ? (n == 0) : (n == nx - 1);
            const int kind = a.fbc[dir < 0 ? 0 : 1];
            if (face && kind != BC_P) return (kind == BC_D ? -1.0 : 1.0) * (double)c[r];
            return (double)(wrap ? t2 : t1);
        } else {
            return 0.0;
        }
    };
    // per-wavefront sums of the source, one record per (batch entry, workgroup, wavefront)
    const int batch = (int)(nblocks / ((size_t)nyb * nz));
    const size_t rec_per_batch = (size_t)gridDim.x * NW;
    if (lane == 0) {
        for (int bb = 0; bb < batch; ++bb) {
            const size_t rec = bb * rec_per_batch + (size_t)blockIdx.x * NW + wave;
            partial[2 * rec] = 0.0;
            partial[2 * rec + 1] = 0.0;
        }
    }
    double acc = 0.0, amax = 0.0;
    int cur_b = -1;
    // RES: the residual's spectra and sums are scaled by a power of two (exact)
    double rscale = 1.0;
    if constexpr (RES) rscale = a.sc[SC_SCALE];
    auto flush = [&]() {
        const double s_ = wave_sum(acc) * rscale, m_ = wave_max(amax) * rscale;
        if (lane == 0 && cur_b >= 0) {
            const size_t rec = cur_b * rec_per_batch + (size_t)blockIdx.x * NW + wave;
            partial[2 * rec] = s_;
            partial[2 * rec + 1] = m_;
        }
        acc = 0.0;
        amax = 0.0;
    };
    // post-processed spectral pair (rows ya, ya+1) of slot m from line j
    auto column = [&](int m, int j, cplx<T>& oa, cplx<T>& ob) {
        const cplx<T>* line = lds + j * ldl;
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
            const cplx<T> c0 = dct_bin<T>(line, mkl, k0, nx);
            const cplx<T> c1 = (FULL || k1 < nx) ? dct_bin<T>(line, mkl, k1, nx) : mk<T>(T(0), T(0));
            oa = mk<T>(c0.x, c1.x);
            ob = mk<T>(c0.y, c1.y);
        }
    };

    auto step = [&](int blk) {
        const XBlock xb = x_block(blk, nyb, nz, ty);
        if (xb.b != cur_b) {
            flush();
            cur_b = xb.b;
        }
        fetch_nb(blk);
        lds_barrier();   // the previous column writes are done reading the lines (and the twiddles are in)
        cplx<T> vf[R512 ? 8 : 1];   // periodic rows of 512: the packed line stays in registers
        // 1. registers -> own packed lines (row 2j real part, row 2j+1 imaginary part),
        //    pre-processed for the x transform; face values lifted into the source;
        //    wavefront sums of the (lifted) source
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int p = FULL ? 0 : fdiv(r, inv_epl);
            const int j = wave + NW * p, n = lane + 64 * (r - p * epl);
            if (FULL || (j < nlines && n < nx)) {
                double la = 0.0, lb = 0.0;   // x-face lift of rows ya, ya + 1 at column n (FULL)
                if constexpr (FACES && FULL) {
                    if (n == 0) {
                        la += fa.c[0] * (double)gx[0];
                        lb += fa.c[0] * (double)gx[1];
                    }
                    if (n == nx - 1) {
                        la += fa.c[1] * (double)gx[2];
                        lb += fa.c[1] * (double)gx[3];
                    }
                }
                double fa_ = (double)ra[r] - la, fb_ = (double)rb[r] - lb;
                if constexpr (RES) {
                    // r = f - lift - c - L_h u0; second differences as sums of first
                    // differences (as in k_residual)
                    const int ya = xb.y0 + 2 * j;
                    const bool va = FULL || ya < ny, vb = FULL || ya + 1 < ny;
                    const double ca = ua[r], cb = ub[r];
                    double xam, xap, xbm, xbp;
                    if constexpr (FULL) {
                        xam = xnb(ua, r, -1);
                        xap = xnb(ua, r, 1);
                        xbm = xnb(ub, r, -1);
                        xbp = xnb(ub, r, 1);
                    } else {
                        const float* up = a.u0 + ((size_t)xb.b * nz + xb.z) * (size_t)ny * nx;
                        const float* ra_ = up + (size_t)(va ? ya : 0) * nx;
                        const float* rb_ = up + (size_t)(vb ? ya + 1 : 0) * nx;
                        const int qm = nb_idx(n, nx, -1, a.fbc[0]), qp = nb_idx(n, nx, 1, a.fbc[1]);
                        const double sm = nb_sgn(n, nx, -1, a.fbc[0]), sp = nb_sgn(n, nx, 1, a.fbc[1]);
                        xam = va ? sm * (double)ra_[qm] : 0.0;
                        xap = va ? sp * (double)ra_[qp] : 0.0;
                        xbm = vb ? sm * (double)rb_[qm] : 0.0;
                        xbp = vb ? sp * (double)rb_[qp] : 0.0;
                    }
                    const double ya_dn = nb_sgn(ya, ny, -1, a.fbc[2]) * (double)uya[r];
                    const double ya_up = vb ? cb : nb_sgn(ya, ny, 1, a.fbc[3]) * (double)uyb[r];
                    const double yb_up = nb_sgn(ya + 1, ny, 1, a.fbc[3]) * (double)uyb[r];
                    const double sz0 = nb_sgn(xb.z, nz, -1, a.fbc[4]), sz1 = nb_sgn(xb.z, nz, 1, a.fbc[5]);
                    const double lapa = ((xam - ca) + (xap - ca)) * a.ihx2 + ((ya_dn - ca) + (ya_up - ca)) * a.ihy2 +
                                        ((sz0 * (double)uza0[r] - ca) + (sz1 * (double)uza1[r] - ca)) * a.ihz2;
                    const double lapb = ((xbm - cb) + (xbp - cb)) * a.ihx2 + ((ca - cb) + (yb_up - cb)) * a.ihy2 +
                                        ((sz0 * (double)uzb0[r] - cb) + (sz1 * (double)uzb1[r] - cb)) * a.ihz2;
                    double c0 = 0.0;
                    if (a.proj == 1) c0 = a.sc[SC_COUNT + 3 * batch + xb.b];
                    else if (a.proj == 2 && xb.z == 0) c0 = (double)nz * a.sc[SC_COUNT + 3 * batch + xb.b];
                    fa_ = va ? fa_ - c0 - lapa : 0.0;
                    fb_ = vb ? fb_ - c0 - lapb : 0.0;
                }
                acc += fa_ + fb_;
                amax = nmax(amax, nmax(fabs(fa_), fabs(fb_)));
                T va = (T)fa_, vb = (T)fb_;
                int pos = n;
                if (a.bx != BC_P) {
                    pos = makhoul_pos(n, nx);
                    if (a.bx == BC_D && (n & 1)) {
                        va = -va;
                        vb = -vb;
                    }
                }
                if (reg512) vf[R512 ? r : 0] = mk<T>(va, vb);
                else lds[j * ldl + pad(pos)] = mk<T>(va, vb);
            }
        }
        // the remaining face lifts, applied to the lines in place: y and z faces
        // (boundary rows and planes only; FULL) or every face (general form).
        // On the w512 path the line is still in registers (a loop of its own:
        // one shared with the LDS form would make the compiler choose between a
        // register and an LDS address, which moves the registers to memory)
        if constexpr (FACES && R512) {
            if (reg512) {
                const int ya = xb.y0 + 2 * wave;
                if (ya == 0 || ya + 1 == ny - 1 || xb.z == 0 || xb.z == nz - 1) {
#pragma unroll
                    for (int r = 0; r < RMAX; ++r) {
                        const int n = lane + 64 * r;
                        const double la = face_lift_yz(fa, xb.b, n, ya, xb.z, nx, ny, nz);
                        const double lb = face_lift_yz(fa, xb.b, n, ya + 1, xb.z, nx, ny, nz);
                        const double fa_ = (double)vf[r].x - la, fb_ = (double)vf[r].y - lb;
                        acc -= la + lb;
                        amax = nmax(amax, nmax(fabs(fa_), fabs(fb_)));
                        vf[r] = mk<T>((T)fa_, (T)fb_);
                    }
                }
            }
        }
        if constexpr (FACES) {
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (reg512) break;
                const int p = FULL ? 0 : fdiv(r, inv_epl);
                const int j = wave + NW * p, n = lane + 64 * (r - p * epl);
                const int ya = xb.y0 + 2 * j;
                const bool edge = FULL ? (ya == 0 || ya + 1 == ny - 1 || xb.z == 0 || xb.z == nz - 1)
                                       : (j < nlines && n < nx);
                if (edge) {
                    double la = 0.0, lb = 0.0;
                    if constexpr (FULL) {
                        la = face_lift_yz(fa, xb.b, n, ya, xb.z, nx, ny, nz);
                        lb = face_lift_yz(fa, xb.b, n, ya + 1, xb.z, nx, ny, nz);
                    } else {
                        if (ya < ny) la = face_lift(fa, xb.b, n, ya, xb.z, nx, ny, nz);
                        if (ya + 1 < ny) lb = face_lift(fa, xb.b, n, ya + 1, xb.z, nx, ny, nz);
                    }
                    int pos = n;
                    double sg = 1.0;
                    if (a.bx != BC_P) {
                        pos = makhoul_pos(n, nx);
                        if (a.bx == BC_D && (n & 1)) sg = -1.0;
                    }
                    cplx<T>& v = lds[j * ldl + pad(pos)];
                    const double fa_ = sg * (double)v.x - la, fb_ = sg * (double)v.y - lb;
                    acc -= la + lb;
                    amax = nmax(amax, nmax(fabs(fa_), fabs(fb_)));
                    v = mk<T>((T)(sg * fa_), (T)(sg * fb_));
                }
            }
        }
        // the next block's rows (past the end: this block's again, unused)
        const int nxt = x_next_block<false>(blk);
        fetch(nxt < nblocks ? nxt : blk);
        // 2. complex FFT of every own line (FULL: exactly one)
        if (reg512) {
            if constexpr (R512) {
                // first stage on the row registers; the result goes back to the
                // line in natural order for the column writes
                cplx<T>* line = lds + wave * ldl;
                const Tw512Lds<T> tw{twl, lane};
                w512_first<false, T>(vf, line, lane);
                w512_second<false, T>(line, tw, lane);
                w512_last<false, T>(line, tw, lane, vf);
#pragma unroll
                for (int t = 0; t < 8; ++t) line[pad(lane + 64 * t)] = vf[t];
            }
        } else if (FULL) {
            wave_lds_sync();
            wfft<RMAX, false, T>(lds + wave * ldl, a.fx, twl, lane);
        } else {
            for (int j = wave; j < nlines; j += NW) {
                wave_lds_sync();
                wfft<RMAX, false, T>(lds + j * ldl, a.fx, twl, lane);
            }
        }
        lds_barrier();

        // 3. post-process and write columns (y contiguous); one thread per (slot, row pair)
        cplx<Ts>* dstS = S + (size_t)xb.b * a.slots * nz * ny;
        // split store: the slots of the double array take their values unrounded
        auto store = [&](int m, int y, cplx<T> v) {
            if constexpr (RES) v = cscale(v, (T)rscale);
            if constexpr (SPLIT) {
                const int k = m - a.lo0;
                if (k >= 0 && k < a.nlo) {
                    a.slo[(((size_t)xb.b * nz + xb.z) * a.nlo + k) * ny + y] = cvt<double>(v);
                    return;
                }
            }
            // (the float spectra of the double-arithmetic kernel are stored
            // normally: streamed, its launch took 0.47 instead of 0.40 ms at 512^3)
            if constexpr (SPLIT) dstS[(size_t)m * a.sstride + (size_t)xb.z * a.zstride + y] = cvt<Ts>(v);
            else put_spec<Ts>(dstS + (size_t)m * a.sstride + (size_t)xb.z * a.zstride + y, cvt<Ts>(v));
        };
        if (FULL) {
#pragma unroll
            for (int q = 0; q < PAIRS; ++q) {
                const int i = tid + q * NTH;
                const int m = fdiv(i, inv_nl), j = i - m * nlines;
                const int ya = xb.y0 + 2 * j;
                cplx<T> oa, ob;
                column(m, j, oa, ob);
                store(m, ya, oa);
                store(m, ya + 1, ob);
            }
        } else {
            for (int i = tid; i < a.slots * nlines; i += NTH) {
                const int m = fdiv(i, inv_nl), j = i - m * nlines;
                const int ya = xb.y0 + 2 * j, yb = ya + 1;
                cplx<T> oa, ob;
                column(m, j, oa, ob);
                if (ya < ny) store(m, ya, oa);
                if (yb < ny) store(m, yb, ob);
            }
        }
    };
    // the launch grid is small enough that every workgroup's first block exists
    const int first = x_first_block<false>();
    fetch(first);
    step(first);
    for (int blk = x_next_block<false>(first); blk < nblocks; blk = x_next_block<false>(blk)) step(blk);
    flush();
}

// Inverse x transform, persistent like the forward kernel: spectral columns -> rows.
//   periodic  -> complex-to-real inverse DFT, unnormalised (returns N x);
//   DCT / DST -> 2 * DCT-III by the inverse of the reordering scheme
//                (Neumann subsection): W_k = e^{+i pi k/2N} (X_k - i X_{N-k}),
//                X_N = 0, v = IDFT_unnormalised(W), x_{2m} = v_m,
//                x_{2m+1} = v_{N-1-m}; Dirichlet multiplies x_n by (-1)^n
//                (its spectral columns are already stored reversed).
// The gather of the spectral columns reads across lines; the inverse
// transform and the row writes are per wavefront.
// MODE XINV_STORE writes u = x - shift[b]; XINV_UPDATE adds the scaled
// correction to a double u and XINV_FIRST stores it without reading u; both
// write per-wavefront partials (sum over the gauge region, max |d|, max |u|).
// Tp: type of the previous solution an update adds to (Tout: u itself, in
// place; float: the separate array uprev holding the first float solution).
template <typename T, typename Tout, typename Tp, int NTH, int MODE, int RMAX, bool FULL>
__global__ __launch_bounds__(NTH) void k_xinv(const cplx<T>* __restrict__ S, Tout* __restrict__ u,
                                              const Tp* __restrict__ uprev, XArgs<T> a,
                                              const double* __restrict__ shift, const double* __restrict__ scalars,
                                              int gauge_region, double* __restrict__ partial, int nblocks) {
    constexpr bool UPD = (MODE != XINV_STORE);   // refinement update (partials)
    constexpr bool INPLACE = std::is_same_v<Tp, Tout>;
    // rows of 512, double spectra: w512_* stages when x is periodic (in float
    // the extra registers cost more occupancy than the LDS round trip saves)
    constexpr bool R512 = FULL && RMAX == 8 && sizeof(T) == 8;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NW = NTH / 64;
    constexpr int PAIRS = RMAX / 2;    // (slot, row pair) gathers per thread: slots * nlines <= NTH * PAIRS
    const int nx = FULL ? 64 * RMAX : a.nx;
    const int ny = a.ny, nz = a.nz, ty = FULL ? 2 * NW : a.ty, ldl = a.ldl;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nlines = ty >> 1;
    const int nyb = (ny + ty - 1) / ty;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* twl = lds + nlines * ldl;
    cplx<T>* mkl = twl + nx;
    for (int i = tid; i < nx; i += NTH) {
        twl[i] = a.twx[i];
        mkl[i] = a.mkx[i];
    }
    const float inv_nl = 1.0f / (float)nlines;
    const int npair = a.slots * nlines;
    const int batch = (int)(nblocks / ((size_t)nyb * nz));
    const int half = (nx >> 1) + 1;
    double inv_scale = 1.0;
    if (UPD) inv_scale = scalars[SC_INVSCALE];

    // refinement partials, one record per (batch entry, workgroup, wavefront)
    const size_t rec_per_batch = (size_t)gridDim.x * NW;
    if (UPD && lane == 0) {
        for (int bb = 0; bb < batch; ++bb) {
            const size_t rec = bb * rec_per_batch + (size_t)blockIdx.x * NW + wave;
            partial[3 * rec] = 0.0;
            partial[3 * rec + 1] = 0.0;
            partial[3 * rec + 2] = 0.0;
        }
    }
    // dmax, umax by fmax (one instruction; it drops NaN), so a NaN correction is
    // carried by the sum chk into dmax at the flush.  The first solve (XINV_FIRST)
    // needs no maxima: its relative correction is 1 by definition.
    double acc = 0.0, dmax = 0.0, umax = 0.0, chk = 0.0;
    int cur_b = -1;
    auto flush = [&]() {
        if (!UPD) return;
        if (chk != chk) dmax = chk;
        const double s_ = wave_sum(acc), d_ = wave_max(dmax), u_ = wave_max(umax);
        if (lane == 0 && cur_b >= 0) {
            const size_t rec = cur_b * rec_per_batch + (size_t)blockIdx.x * NW + wave;
            partial[3 * rec] = s_;
            partial[3 * rec + 1] = d_;
            partial[3 * rec + 2] = u_;
        }
        acc = 0.0;
        dmax = 0.0;
        umax = 0.0;
        chk = 0.0;
    };

    cplx<T> sa[PAIRS], sb[PAIRS];
    auto fetch = [&](int blk) {
        const XBlock xb = x_block(blk, nyb, nz, ty, a.zends);
        const cplx<T>* srcS = S + (size_t)xb.b * a.slots * nz * ny;
#pragma unroll
        for (int k = 0; k < PAIRS; ++k) {
            const int i = tid + k * NTH;
            if (FULL) {
                const int m = fdiv(i, inv_nl), j = i - m * nlines;
                const int ya = xb.y0 + 2 * j;
                const size_t col = (size_t)m * a.sstride + (size_t)xb.z * a.zstride;
                sa[k] = srcS[col + ya];
                sb[k] = srcS[col + ya + 1];
            } else {
                sa[k] = mk<T>(T(0), T(0));
                sb[k] = sa[k];
                if (i < npair) {
                    const int m = fdiv(i, inv_nl), j = i - m * nlines;
                    const int ya = xb.y0 + 2 * j;
                    const size_t col = (size_t)m * a.sstride + (size_t)xb.z * a.zstride;
                    if (ya < ny) sa[k] = srcS[col + ya];
                    if (ya + 1 < ny) sb[k] = srcS[col + ya + 1];
                }
            }
        }
    };
    // FULL refinement update: the current rows of u for this wave's line, read
    // before the next block's prefetch is issued
    constexpr int UR = (MODE == XINV_UPDATE && FULL) ? 2 * RMAX : 1;
    double uo[UR];
    for (int r = 0; r < UR; ++r) uo[r] = 0.0;

    auto step = [&](int blk) {
        const XBlock xb = x_block(blk, nyb, nz, ty, a.zends);
        if (xb.b != cur_b) {
            flush();
            cur_b = xb.b;
        }
        Tout* dst = u + ((size_t)xb.b * nz + xb.z) * (size_t)ny * nx;
        const Tp* prv = nullptr;
        if constexpr (INPLACE) prv = dst;
        else prv = uprev + ((size_t)xb.b * nz + xb.z) * (size_t)ny * nx;
        lds_barrier();   // the previous inverse transforms are done with the lines (and the twiddles are in)
        // 1. registers -> packed complex spectra of row pairs (any line)
#pragma unroll
        for (int k = 0; k < PAIRS; ++k) {
            const int i = tid + k * NTH;
            if (FULL || i < npair) {
                const int m = fdiv(i, inv_nl), j = i - m * nlines;
                const cplx<T> va = sa[k], vb = sb[k];
                cplx<T>* line = lds + j * ldl;
                if (a.bx == BC_P) {
                    if (m == 0) {
                        line[pad(0)] = mk<T>(va.x, vb.x);
                        if (!(nx & 1)) line[pad(nx >> 1)] = mk<T>(va.y, vb.y);
                    } else {
                        line[pad(m)] = mk<T>(va.x - vb.y, va.y + vb.x);        // X_a + i X_b
                        line[pad(nx - m)] = mk<T>(va.x + vb.y, vb.x - va.y);   // conj(X_a) + i conj(X_b)
                    }
                } else {
                    line[pad(2 * m)] = mk<T>(va.x, vb.x);
                    if (FULL || 2 * m + 1 < nx) line[pad(2 * m + 1)] = mk<T>(va.y, vb.y);
                }
            }
        }
        if (MODE == XINV_UPDATE && FULL) {
#pragma unroll
            for (int k = 0; k < RMAX; ++k)
#pragma unroll
                for (int part = 0; part < 2; ++part)
                    uo[2 * k + part] = (double)prv[(size_t)(xb.y0 + 2 * wave + part) * nx + lane + 64 * k];
        }
        // the next block's spectra (past the end: this block's again, unused)
        const int nxt = x_next_block<sizeof(T) == 4>(blk);   // pairs in float (x_next_block)
        fetch(nxt < nblocks ? nxt : blk);
        lds_barrier();

        const double sh = shift ? shift[xb.b] : 0.0;
        double gshift = 0.0;
        if (UPD) gshift = scalars[SC_COUNT + 2 * batch + xb.b];
        // 2. per own line (FULL: exactly one): inverse pre-processing, inverse FFT, row writes
        for (int j = wave; FULL ? j == wave : j < nlines; j += NW) {
            cplx<T>* line = lds + j * ldl;
            if (a.bx != BC_P) {
                for (int k = lane; k < half; k += 64) {
                    if (k == 0) continue;                       // W_0 = X_0
                    const cplx<T> xk = line[pad(k)];
                    if (2 * k == nx) {
                        line[pad(k)] = cmulc(mk<T>(xk.x + xk.y, xk.y - xk.x), mkl[k]);   // e^{+} (X_k - i X_k)
                    } else {
                        const cplx<T> xr = line[pad(nx - k)];
                        // X_k - i X_{N-k} = (xk.x + xr.y, xk.y - xr.x)
                        line[pad(k)] = cmulc(mk<T>(xk.x + xr.y, xk.y - xr.x), mkl[k]);
                        line[pad(nx - k)] = cmulc(mk<T>(xr.x + xk.y, xr.y - xk.x), mkl[nx - k]);
                    }
                }
            }
            wave_lds_sync();
            // periodic rows of 512: the last stage's outputs stay in registers,
            // in the order the row writes take them (see w512_last)
            cplx<T> vl[R512 ? 8 : 1];
            if constexpr (R512) {
                if (a.bx == BC_P) {
                    const Tw512Lds<T> tw{twl, lane};
                    w512_first_lds<true, T>(line, lane);
                    w512_second<true, T>(line, tw, lane);
                    w512_last<true, T>(line, tw, lane, vl);
                } else {
                    wfft<RMAX, true, T>(line, a.fx, twl, lane);
                }
            } else {
                wfft<RMAX, true, T>(line, a.fx, twl, lane);
            }
            if (FULL) {
#pragma unroll
                for (int k = 0; k < RMAX; ++k) {
                    const int n = lane + 64 * k;
                    int pos = n;
                    if (a.bx != BC_P) pos = makhoul_pos(n, nx);
                    cplx<T> c;
                    if constexpr (R512) c = (a.bx == BC_P) ? vl[k] : line[pad(pos)];
                    else c = line[pad(pos)];
                    if (a.bx == BC_D && (n & 1)) c = mk<T>(-c.x, -c.y);
#pragma unroll
                    for (int part = 0; part < 2; ++part) {
                        const int y = xb.y0 + 2 * j + part;
                        const T v = part ? c.y : c.x;
                        const size_t idx = (size_t)y * nx + n;
                        if (MODE == XINV_STORE) {
                            st_stream(dst + idx, (Tout)((double)v - sh));
                        } else {
                            const double d = ((double)v - sh) * inv_scale;
                            // uo = 0 for XINV_FIRST; sums and maxima of the stored value
                            const double un = (double)(Tout)(uo[UR > 1 ? 2 * k + part : 0] + d - gshift);
                            st_stream(dst + idx, (Tout)un);
                            if (gauge_region == 1 || (gauge_region == 2 && xb.z == 0)) acc += un;
                            if constexpr (MODE == XINV_UPDATE) {
                                dmax = fmax(dmax, fabs(d));
                                umax = fmax(umax, fabs(un));
                                chk += d;
                            }
                        }
                    }
                }
            } else {
                for (int n = lane; n < nx; n += 64) {
                    int pos = n;
                    if (a.bx != BC_P) pos = makhoul_pos(n, nx);
                    cplx<T> c = line[pad(pos)];
                    if (a.bx == BC_D && (n & 1)) c = mk<T>(-c.x, -c.y);
#pragma unroll
                    for (int part = 0; part < 2; ++part) {
                        const int y = xb.y0 + 2 * j + part;
                        if (y >= ny) continue;
                        const T v = part ? c.y : c.x;
                        const size_t idx = (size_t)y * nx + n;
                        if (MODE == XINV_STORE) {
                            st_stream(dst + idx, (Tout)((double)v - sh));
                        } else {
                            const double d = ((double)v - sh) * inv_scale;
                            const double un = (double)(Tout)((MODE == XINV_UPDATE ? (double)prv[idx] : 0.0) + d - gshift);
                            st_stream(dst + idx, (Tout)un);
                            if (gauge_region == 1 || (gauge_region == 2 && xb.z == 0)) acc += un;
                            if constexpr (MODE == XINV_UPDATE) {
                                dmax = fmax(dmax, fabs(d));
                                umax = fmax(umax, fabs(un));
                                chk += d;
                            }
                        }
                    }
                }
            }
        }
    };
    // the launch grid is small enough that every workgroup's first block exists
    constexpr bool PAIR = sizeof(T) == 4;
    const int first = x_first_block<PAIR>();
    fetch(first);
    step(first);
    for (int blk = x_next_block<PAIR>(first); blk < nblocks; blk = x_next_block<PAIR>(blk)) step(blk);
    flush();
}

template <typename T> static size_t x_lds_bytes(const XArgs<T>& a) {
    return ((size_t)(a.ty >> 1) * a.ldl + 2 * (size_t)a.nx) * sizeof(cplx<T>);
}

hipError_t allow_dynamic_lds(const void* kernel, int bytes) {
    static std::mutex mu;
    static std::set<std::tuple<const void*, int, int>> done;   // (kernel, device, bytes)
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count({kernel, dev, bytes})) return hipSuccess;
    const hipError_t r = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (r == hipSuccess) done.insert({kernel, dev, bytes});
    return r;
}

// Allow the kernel the dynamic LDS it may ask for (lines + twiddle tables)
// (the template argument is the kernel itself).
template <auto K> static hipError_t allow_lds() {
    return allow_dynamic_lds(reinterpret_cast<const void*>(K), kXLdsMax);
}

int device_cus() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    return cus;
}

// Persistent grid: a few resident workgroups per CU.
int x_grid(int nblocks) {
    const int cus = device_cus();
    return nblocks < cus * kXBlocksPerCU ? nblocks : cus * kXBlocksPerCU;
}

int x_blocks(int ny, int ty, int nz, int batch) { return ((ny + ty - 1) / ty) * nz * batch; }

int x_launch_grid(int nblocks, bool paired) { return x_grid(paired ? (nblocks + 1) / 2 : nblocks); }

// Row blocks of the FULL shape: nx = 64 RMAX, one line per wavefront, whole blocks
// in y.  Lines of 2048 never fit four to a workgroup, so RMAX = 32 has no FULL form.
template <int RMAX, typename T> static bool x_full(const XArgs<T>& a) {
    return RMAX <= 16 && a.nx == 64 * RMAX && a.ty == 2 * kXWaves && a.ny % a.ty == 0;
}

template <typename T, typename Tin, typename Ts, int RMAX, bool FACES, bool RES = false>
static hipError_t launch_xfwd_shape(const Tin* f, cplx<Ts>* S, double* partial, const XArgs<T>& a, int batch,
                                    const FaceArgs<Tin>& fa, hipStream_t s) {
    const int nb = x_blocks(a.ny, a.ty, a.nz, batch);
    if constexpr (RMAX <= 16) {
        if (x_full<RMAX>(a)) {
            const hipError_t le = allow_lds<k_xfwd<T, Tin, Ts, kXThreads, RMAX, true, FACES, RES>>();
            if (le != hipSuccess) return le;
            hipLaunchKernelGGL((k_xfwd<T, Tin, Ts, kXThreads, RMAX, true, FACES, RES>),
                               dim3(x_launch_grid(nb, false)), dim3(kXThreads), x_lds_bytes(a), s, f, S, partial, a,
                               nb, fa);
            return hipGetLastError();
        }
    }
    {
        const hipError_t le = allow_lds<k_xfwd<T, Tin, Ts, kXThreads, RMAX, false, FACES, RES>>();
        if (le != hipSuccess) return le;
        hipLaunchKernelGGL((k_xfwd<T, Tin, Ts, kXThreads, RMAX, false, FACES, RES>), dim3(x_launch_grid(nb, false)),
                           dim3(kXThreads), x_lds_bytes(a), s, f, S, partial, a, nb, fa);
    }
    return hipGetLastError();
}

bool res_fused_supported(int nx) { return nx <= 512; }

hipError_t launch_xfwd_res(const double* f, cplx<float>* S, double* partial, const XArgs<double>& a, int batch,
                           const FaceArgs<double>* faces, hipStream_t s) {
    if (a.nx > 512) return hipErrorInvalidValue;
    const FaceArgs<double> none{};
    if (faces) {
        if (a.nx == 256) return launch_xfwd_shape<double, double, float, 4, true, true>(f, S, partial, a, batch, *faces, s);
        if (a.nx == 384) return launch_xfwd_shape<double, double, float, 6, true, true>(f, S, partial, a, batch, *faces, s);
        return launch_xfwd_shape<double, double, float, 8, true, true>(f, S, partial, a, batch, *faces, s);
    }
    if (a.nx == 256) return launch_xfwd_shape<double, double, float, 4, false, true>(f, S, partial, a, batch, none, s);
    if (a.nx == 384) return launch_xfwd_shape<double, double, float, 6, false, true>(f, S, partial, a, batch, none, s);
    return launch_xfwd_shape<double, double, float, 8, false, true>(f, S, partial, a, batch, none, s);
}

template <typename T, typename Tin, typename Ts, bool FACES>
static hipError_t launch_xfwd_any(const Tin* f, cplx<Ts>* S, double* partial, const XArgs<T>& a, int batch,
                                  const FaceArgs<Tin>& fa, hipStream_t s) {
    // rows of 256 = 64 x 4 and 384 = 64 x 6: exact-count forms with four and
    // six values per lane
    if (a.nx == 256) return launch_xfwd_shape<T, Tin, Ts, 4, FACES>(f, S, partial, a, batch, fa, s);
    if (a.nx == 384) return launch_xfwd_shape<T, Tin, Ts, 6, FACES>(f, S, partial, a, batch, fa, s);
    if (a.nx <= 512) return launch_xfwd_shape<T, Tin, Ts, 8, FACES>(f, S, partial, a, batch, fa, s);
    if (a.nx <= 1024) return launch_xfwd_shape<T, Tin, Ts, 16, FACES>(f, S, partial, a, batch, fa, s);
    return launch_xfwd_shape<T, Tin, Ts, 32, FACES>(f, S, partial, a, batch, fa, s);
}

template <typename T, typename Tin, typename Ts>
hipError_t launch_xfwd(const Tin* f, cplx<Ts>* S, double* partial, const XArgs<T>& a, int batch,
                       const FaceArgs<Tin>* faces, hipStream_t s) {
    if (faces) return launch_xfwd_any<T, Tin, Ts, true>(f, S, partial, a, batch, *faces, s);
    const FaceArgs<Tin> none{};
    return launch_xfwd_any<T, Tin, Ts, false>(f, S, partial, a, batch, none, s);
}

template <typename T, typename Tout, typename Tp, int MODE, int RMAX>
static hipError_t launch_xinv_shape(const cplx<T>* S, Tout* u, const Tp* uprev, const XArgs<T>& a, int batch,
                                    const double* shift, const double* scalars, int gauge_region, double* partial,
                                    hipStream_t s) {
    const int nb = x_blocks(a.ny, a.ty, a.nz, batch);
    if constexpr (RMAX <= 16) {
        if (x_full<RMAX>(a)) {
            const hipError_t le = allow_lds<k_xinv<T, Tout, Tp, kXThreads, MODE, RMAX, true>>();
            if (le != hipSuccess) return le;
            hipLaunchKernelGGL((k_xinv<T, Tout, Tp, kXThreads, MODE, RMAX, true>),
                               dim3(x_launch_grid(nb, sizeof(T) == 4)), dim3(kXThreads), x_lds_bytes(a), s, S, u,
                               uprev, a, shift, scalars, gauge_region, partial, nb);
            return hipGetLastError();
        }
    }
    {
        const hipError_t le = allow_lds<k_xinv<T, Tout, Tp, kXThreads, MODE, RMAX, false>>();
        if (le != hipSuccess) return le;
        hipLaunchKernelGGL((k_xinv<T, Tout, Tp, kXThreads, MODE, RMAX, false>),
                           dim3(x_launch_grid(nb, sizeof(T) == 4)), dim3(kXThreads), x_lds_bytes(a), s, S, u, uprev,
                           a, shift, scalars, gauge_region, partial, nb);
    }
    return hipGetLastError();
}

template <typename T, typename Tout, typename Tp, int MODE>
static hipError_t launch_xinv_any(const cplx<T>* S, Tout* u, const Tp* uprev, const XArgs<T>& a, int batch,
                                  const double* shift, const double* scalars, int gauge_region, double* partial,
                                  hipStream_t s) {
    if (a.nx == 256)   // 64 x 4: exact-count form with four values per lane
        return launch_xinv_shape<T, Tout, Tp, MODE, 4>(S, u, uprev, a, batch, shift, scalars, gauge_region, partial, s);
    if (a.nx == 384)   // 64 x 6: exact-count form with six values per lane
        return launch_xinv_shape<T, Tout, Tp, MODE, 6>(S, u, uprev, a, batch, shift, scalars, gauge_region, partial, s);
    if (a.nx <= 512)
        return launch_xinv_shape<T, Tout, Tp, MODE, 8>(S, u, uprev, a, batch, shift, scalars, gauge_region, partial, s);
    if (a.nx <= 1024)
        return launch_xinv_shape<T, Tout, Tp, MODE, 16>(S, u, uprev, a, batch, shift, scalars, gauge_region, partial,
                                                        s);
    return launch_xinv_shape<T, Tout, Tp, MODE, 32>(S, u, uprev, a, batch, shift, scalars, gauge_region, partial, s);
}

template <typename T, typename Tout>
hipError_t launch_xinv(const cplx<T>* S, Tout* u, const XArgs<T>& a, int batch, const double* shift, hipStream_t s) {
    return launch_xinv_any<T, Tout, Tout, XINV_STORE>(S, u, (const Tout*)nullptr, a, batch, shift,
                                                      (const double*)nullptr, 0, (double*)nullptr, s);
}

hipError_t launch_xinv_first(const cplx<float>* S, float* u0, const XArgs<float>& a, int batch, const double* scalars,
                             int gauge_region, double* partial, hipStream_t s) {
    // no mean shift: u0 holds the transform's own float values, so storing it
    // rounds nothing; the gauge shift of the first update removes the mean
    return launch_xinv_any<float, float, float, XINV_FIRST>(S, u0, (const float*)nullptr, a, batch,
                                                            (const double*)nullptr, scalars, gauge_region, partial, s);
}

hipError_t launch_xinv_update(const cplx<float>* S, double* u, const float* uprev, const XArgs<float>& a, int batch,
                              const double* scalars, int gauge_region, double* partial, int mode, hipStream_t s) {
    const double* shift = scalars + SC_COUNT + batch;   // cmean of the correction solve
    if (mode == XINV_FIRST)
        return launch_xinv_any<float, double, double, XINV_FIRST>(S, u, (const double*)nullptr, a, batch, shift,
                                                                  scalars, gauge_region, partial, s);
    if (uprev)
        return launch_xinv_any<float, double, float, XINV_UPDATE>(S, u, uprev, a, batch, shift, scalars,
                                                                  gauge_region, partial, s);
    return launch_xinv_any<float, double, double, XINV_UPDATE>(S, u, (const double*)nullptr, a, batch, shift, scalars,
                                                               gauge_region, partial, s);
}

template hipError_t launch_xfwd<double, double, double>(const double*, cplx<double>*, double*, const XArgs<double>&,
                                                        int, const FaceArgs<double>*, hipStream_t);
template hipError_t launch_xfwd<float, float, float>(const float*, cplx<float>*, double*, const XArgs<float>&, int,
                                                     const FaceArgs<float>*, hipStream_t);
// refined solve: double arithmetic, float spectra (and the double slots)
template hipError_t launch_xfwd<double, double, float>(const double*, cplx<float>*, double*, const XArgs<double>&,
                                                       int, const FaceArgs<double>*, hipStream_t);
template hipError_t launch_xfwd<double, float, float>(const float*, cplx<float>*, double*, const XArgs<double>&, int,
                                                      const FaceArgs<float>*, hipStream_t);
template hipError_t launch_xinv<double, double>(const cplx<double>*, double*, const XArgs<double>&, int,
                                                const double*, hipStream_t);
template hipError_t launch_xinv<float, float>(const cplx<float>*, float*, const XArgs<float>&, int, const double*,
                                              hipStream_t);

}  // namespace pp
