// Alternative z solvers: parallel cyclic reduction (section "Parallel Cyclic
// Reduction") and cyclic reduction with a parallel backward phase (section
// "Cyclic Reduction Technique", CR-P).  Selected per plan; the default is the
// fused Thomas march.
//
// Both need a whole z line of a mode on chip at once, while the y transform
// needs a whole y line of a plane, so this path runs them as separate passes
// over the spectral array S:
//   k_ypass<FWD>     y transform of every (slot, plane), in place;
//   k_zpcr / k_zcr   PCR / CR-P along z for tiles of real systems (the parts of
//                    entries) of one slot, the whole line of each in LDS;
//   k_ypass<INV>     inverse y transform, in place.
// Two more HBM sweeps than the fused march (the point of the comparison).
//
// PCR on the normalised system (diagonal 1): row j reads
//     a_j u_{j-1} + u_j + c_j u_{j+1} = x_j,
// and one level with stride s replaces it by a combination of rows j-s, j, j+s:
//     r = 1 / (1 - a_j c_{j-s} - c_j a_{j+s})
//     a_j <- -r a_j a_{j-s},  c_j <- -r c_j c_{j+s},
//     x_j <- r (x_j - a_j x_{j-s} - c_j x_{j+s}),
// with rows outside [0, n) taken as zero.  After ceil(log2 n) levels every row
// is decoupled and x_j = u_j.  Every row of a level reads the old values of
// its neighbours: the level reads into registers, then writes back after a
// barrier.  The zero mode of a singular problem is pinned (row 0: u_0 = 0).

#include "pp_kernels.hpp"

namespace pp {

// ---------------------------------------------------------------- y passes
// One 512-thread workgroup per (slot, 8 planes, batch entry); one plane per
// wavefront, transformed in a padded LDS line with the wavefront-private FFT.
template <typename T, bool INV>
__global__ __launch_bounds__(512) void k_ypass(cplx<T>* __restrict__ S, MidArgs<T> a) {
    constexpr int LDY = 576;
    __shared__ __align__(16) cplx<T> work[8 * LDY];
    __shared__ __align__(16) cplx<T> twl[512];
    __shared__ __align__(16) cplx<T> mkl[512];
    const int m = blockIdx.x, b = blockIdx.z;
    const int ny = a.ny, nz = a.nz;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int i = tid; i < ny; i += 512) {
        twl[i] = a.twy[i];
        mkl[i] = a.mky[i];
    }
    __syncthreads();
    const int z = blockIdx.y * 8 + wave;
    if (z >= nz) return;
    const bool pairslot = (a.bx != BC_P) || (m == 0);
    const bool sep = (a.by == BC_P) && pairslot;
    const int half = (ny >> 1) + 1;
    cplx<T>* plane = S + (size_t)b * a.slots * nz * ny + (size_t)m * a.sstride + (size_t)z * a.zstride;
    cplx<T>* line = work + wave * LDY;
    if (!INV) {
        for (int y = lane; y < ny; y += 64) {
            cplx<T> v = plane[y];
            int pos = y;
            if (a.by != BC_P) {
                pos = makhoul_pos(y, ny);
                if (a.by == BC_D && (y & 1)) v = mk<T>(-v.x, -v.y);
            }
            line[pad(pos)] = v;
        }
        wave_lds_sync();
        wfft<8, false, T>(line, a.fy, twl, lane);
        if (a.by != BC_P) {
            for (int k = lane; k < half; k += 64) {
                if (k == 0) continue;
                const cplx<T> vk = line[pad(k)];
                const cplx<T> wk = mkl[k];
                if (2 * k == ny) {
                    line[pad(k)] = cscale(cadd(cmul(wk, vk), cmulc(vk, wk)), T(0.5));
                } else {
                    const cplx<T> vr = line[pad(ny - k)];
                    const cplx<T> wr = mkl[ny - k];
                    line[pad(k)] = cscale(cadd(cmul(wk, vk), cmulc(vr, wk)), T(0.5));
                    line[pad(ny - k)] = cscale(cadd(cmul(wr, vr), cmulc(vk, wr)), T(0.5));
                }
            }
        } else if (sep) {
            for (int k = lane; k < half; k += 64) {
                if (k == 0 || 2 * k >= ny) continue;
                const cplx<T> zk = line[pad(k)], zr = line[pad(ny - k)];
                line[pad(k)] = mk<T>(T(0.5) * (zk.x + zr.x), T(0.5) * (zk.y - zr.y));
                line[pad(ny - k)] = mk<T>(T(0.5) * (zk.y + zr.y), T(0.5) * (zr.x - zk.x));
            }
        }
        wave_lds_sync();
        for (int e = lane; e < ny; e += 64) plane[e] = line[pad(e)];
    } else {
        for (int e = lane; e < ny; e += 64) line[pad(e)] = plane[e];
        wave_lds_sync();
        if (a.by != BC_P) {
            for (int k = lane; k < half; k += 64) {
                if (k == 0) continue;
                const cplx<T> xk = line[pad(k)];
                if (2 * k == ny) {
                    line[pad(k)] = cmulc(mk<T>(xk.x + xk.y, xk.y - xk.x), mkl[k]);
                } else {
                    const cplx<T> xr = line[pad(ny - k)];
                    line[pad(k)] = cmulc(mk<T>(xk.x + xr.y, xk.y - xr.x), mkl[k]);
                    line[pad(ny - k)] = cmulc(mk<T>(xr.x + xk.y, xr.y - xk.x), mkl[ny - k]);
                }
            }
        } else if (sep) {
            for (int k = lane; k < half; k += 64) {
                if (k == 0 || 2 * k >= ny) continue;
                const cplx<T> A = line[pad(k)], B = line[pad(ny - k)];
                line[pad(k)] = mk<T>(A.x - B.y, A.y + B.x);
                line[pad(ny - k)] = mk<T>(A.x + B.y, B.x - A.y);
            }
        }
        wave_lds_sync();
        wfft<8, true, T>(line, a.fy, twl, lane);
        for (int y = lane; y < ny; y += 64) {
            int pos = y;
            if (a.by != BC_P) pos = makhoul_pos(y, ny);
            cplx<T> v = line[pad(pos)];
            if (a.by == BC_D && (y & 1)) v = mk<T>(-v.x, -v.y);
            plane[y] = v;
        }
    }
}

// ------------------------------------------------ PCR and CR-P along z
// The real and imaginary parts of an entry are independent systems.  Lines up
// to 2048 rows use the paired layout below (k_zpcr2, k_zcr2); longer ones, up
// to 4096, a 256-thread workgroup per real system ("part": part p of the tile
// is entry e0 + p / 2, component p % 2; TP parts per tile, TP = 1 there), the
// whole z line in LDS: per (z, part) the right-hand side x and the two
// off-diagonals a, c (24 B, 98 KB at 4096 rows).  The
// reductions run in double for either solve precision: their log2(nz) levels
// of combined rows lose more to rounding than the Thomas recurrence does,
// which in float exceeds the unrefined float tolerance on long lines.
constexpr int kPcrThreads = 256;
constexpr int kPcrPairRows = 2048;           // nz * TE per workgroup, paired layout
constexpr int kPcrRowsMax = 4096;            // nz * TP per workgroup
constexpr int kPcrItems = kPcrRowsMax / kPcrThreads;   // rows per thread (PCR registers)
int pcr_parts(int nz) {
    int tp = 8;
    while (tp > 1 && nz * tp > kPcrRowsMax) tp >>= 1;
    return tp;
}
size_t pcr_lds_bytes(int nz) { return (size_t)nz * pcr_parts(nz) * 3 * sizeof(double) + 64 * sizeof(double); }
// paired layout: entries per tile (0: the line is too long for it)
int pcr_entries(int nz) {
    int te = 4;
    while (te > 0 && nz * te > kPcrPairRows) te >>= 1;
    return te;
}
size_t pcr2_lds_bytes(int nz) {
    return (size_t)nz * pcr_entries(nz) * (sizeof(double2) + 4 * sizeof(double)) + 64 * sizeof(double);
}

// Load the tile's z lines of slot m into LDS (row r = z * TP + p), scaled and
// normalised to a unit diagonal; the zero mode pinned (row 0: u_0 = 0, row 1
// without its coupling to u_0).
template <typename Tio>
__device__ void tri_load(const cplx<Tio>* __restrict__ S, const MidArgs<Tio>& a, size_t base, int m, int b, int p0,
                         int tp, double* X, double* A, double* C) {
    using T = double;
    const int nz = a.nz, ny = a.ny;
    const bool sing = a.singular && m == 0;
    const T proj = (sing && a.project) ? (T)(a.hz2 * a.mu[b]) : T(0);
    const T d0 = (a.bz0 == BC_D) ? T(-1) : T(1), d1 = (a.bz1 == BC_D) ? T(-1) : T(1);
    // tp even: a thread reads one complex value and fills both parts' rows
    const int cp = (tp & 1) ? 1 : 2;
    const int nitems = nz * tp / cp;
    for (int it = threadIdx.x; it < nitems; it += kPcrThreads)
    for (int c2 = 0; c2 < cp; ++c2) {
        const int r = it * cp + c2;
        const int z = r / tp, pl = r - z * tp, pg = p0 + pl;
        const int e = pg >> 1, comp = pg & 1;
        T x = T(0), bm = T(1);
        if (e < ny) {
            const cplx<Tio> xs = S[base + (size_t)z * a.zstride + e];
            const cplx<Tio> bs = a.bmid[(size_t)m * ny + e];
            x = (T)(comp ? xs.y : xs.x) * (T)a.scale;
            bm = (T)(comp ? bs.y : bs.x);
        }
        const bool pin = sing && e == 0 && comp == 0;   // the zero mode: row 0 reads u_0 = 0
        if (pin) x -= proj;
        T bd = bm;
        if (z == 0) bd += d0;
        if (z == nz - 1) bd += d1;
        if (nz == 1) bd = bm + d0 + d1;
        const T ib = T(1) / bd;
        T av = (z > 0) ? ib : T(0);
        T cv = (z < nz - 1) ? ib : T(0);
        T xv = x * ib;
        if (pin && z == 0) {
            av = cv = T(0);
            xv = T(0);
        }
        if (pin && z == 1) av = T(0);   // coupling to the pinned u_0 = 0
        X[r] = xv;
        A[r] = av;
        C[r] = cv;
    }
}

// Store the solved lines (each part into its component); the mean of the
// zero-mode line for the zero-mean gauge.
template <typename Tio>
__device__ void tri_store(cplx<Tio>* __restrict__ S, const MidArgs<Tio>& a, size_t base, int m, int b, int p0,
                          int tp, const double* X, double* red) {
    const int nz = a.nz, ny = a.ny;
    const bool sing = a.singular && m == 0;
    double csum = 0.0;
    if (!(tp & 1)) {
        // whole complex values: parts 2q, 2q + 1 of a row are the entry's two components
        for (int it = threadIdx.x; it < nz * tp / 2; it += kPcrThreads) {
            const int r = 2 * it;
            const int z = r / tp, pl = r - z * tp, e = (p0 + pl) >> 1;
            if (e >= ny) continue;
            S[base + (size_t)z * a.zstride + e] = mk<Tio>((Tio)X[r], (Tio)X[r + 1]);
            if (sing && e == 0) csum += X[r];
        }
    } else {
        Tio* Sr = reinterpret_cast<Tio*>(S);
        for (int r = threadIdx.x; r < nz * tp; r += kPcrThreads) {
            const int z = r / tp, pl = r - z * tp, pg = p0 + pl;
            const int e = pg >> 1, comp = pg & 1;
            if (e >= ny) continue;
            const double u = X[r];
            Sr[2 * (base + (size_t)z * a.zstride + e) + comp] = (Tio)u;
            if (sing && e == 0 && comp == 0) csum += u;
        }
    }
    if (m == 0 && blockIdx.x == 0) {
        const double tot = block_sum<kPcrThreads>(csum, red);
        if (threadIdx.x == 0) a.cmean[b] = (sing && a.demean) ? tot / (double)nz : 0.0;
    }
}

template <typename Tio>
__global__ __launch_bounds__(kPcrThreads) void k_zpcr(cplx<Tio>* __restrict__ S, MidArgs<Tio> a, int tp) {
    using T = double;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nz = a.nz;
    const int m = blockIdx.y, b = blockIdx.z;
    const int p0 = blockIdx.x * tp;
    const int tid = threadIdx.x;
    const int nrows = nz * tp;
    T* X = reinterpret_cast<T*>(smem);     // [z][tp]
    T* A = X + nrows;
    T* C = A + nrows;
    double* red = C + nrows;
    const size_t base = (size_t)b * a.slots * nz * a.ny + (size_t)m * a.sstride;
    tri_load<Tio>(S, a, base, m, b, p0, tp, X, A, C);
    __syncthreads();
    for (int s = 1; s < nz; s <<= 1) {
        T nx_[kPcrItems], na[kPcrItems], nc[kPcrItems];
#pragma unroll
        for (int k = 0; k < kPcrItems; ++k) {
            const int r = tid + k * kPcrThreads;
            if (r >= nrows) continue;
            const int z = r / tp;
            T am = T(0), cm = T(0), xm = T(0), ap = T(0), cp = T(0), xp = T(0);
            if (z - s >= 0) {
                am = A[r - s * tp];
                cm = C[r - s * tp];
                xm = X[r - s * tp];
            }
            if (z + s < nz) {
                ap = A[r + s * tp];
                cp = C[r + s * tp];
                xp = X[r + s * tp];
            }
            const T ar = A[r], cr = C[r];
            const T rr = T(1) / (T(1) - ar * cm - cr * ap);
            na[k] = -rr * ar * am;
            nc[k] = -rr * cr * cp;
            nx_[k] = rr * (X[r] - ar * xm - cr * xp);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPcrItems; ++k) {
            const int r = tid + k * kPcrThreads;
            if (r >= nrows) continue;
            A[r] = na[k];
            C[r] = nc[k];
            X[r] = nx_[k];
        }
        __syncthreads();
    }
    tri_store<Tio>(S, a, base, m, b, p0, tp, X, red);
}

// Cyclic reduction with a parallel backward phase (section "Cyclic Reduction
// Technique", CR-P).  Forward: at stride s = 1, 2, 4, ... (while 2s <= nz) the
// rows z = 2s-1, 4s-1, ... are combined with rows z -+ s as in PCR,
//     r = 1 / (1 - a_z c_{z-s} - c_z a_{z+s})
//     a_z <- -r a_z a_{z-s},  c_z <- -r c_z c_{z+s},
//     x_z <- r (x_z - a_z x_{z-s} - c_z x_{z+s}),
// which leaves them coupled to rows z -+ 2s only; the rows a level reads are
// not the rows it writes, so a level needs one barrier.  The last stride s
// leaves the single row s-1, already decoupled (x = u).  Backward: for
// t = s/2, ..., 1 the rows z = t-1, 3t-1, ... take u_z = x_z - a_z u_{z-t} -
// c_z u_{z+t}, their neighbours being solved at the coarser levels.  Rows
// outside [0, nz) count as zero.
template <typename Tio>
__global__ __launch_bounds__(kPcrThreads) void k_zcr(cplx<Tio>* __restrict__ S, MidArgs<Tio> a, int tp) {
    using T = double;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nz = a.nz;
    const int m = blockIdx.y, b = blockIdx.z;
    const int p0 = blockIdx.x * tp;
    const int tid = threadIdx.x;
    const int nrows = nz * tp;
    T* X = reinterpret_cast<T*>(smem);     // [z][tp]
    T* A = X + nrows;
    T* C = A + nrows;
    double* red = C + nrows;
    const size_t base = (size_t)b * a.slots * nz * a.ny + (size_t)m * a.sstride;
    tri_load<Tio>(S, a, base, m, b, p0, tp, X, A, C);
    __syncthreads();
    int s = 1;
    for (; 2 * s <= nz; s <<= 1) {
        const int cnt = (nz - (2 * s - 1) + 2 * s - 1) / (2 * s);   // rows 2s-1 + 2s q < nz
        for (int w = tid; w < cnt * tp; w += kPcrThreads) {
            const int q = w / tp, pl = w - q * tp;
            const int z = 2 * s - 1 + 2 * s * q;
            const int r = z * tp + pl;
            const T am = A[r - s * tp], cm = C[r - s * tp], xm = X[r - s * tp];   // z - s >= s - 1 >= 0
            T ap = T(0), cp = T(0), xp = T(0);
            if (z + s < nz) {
                ap = A[r + s * tp];
                cp = C[r + s * tp];
                xp = X[r + s * tp];
            }
            const T ar = A[r], cr = C[r];
            const T rr = T(1) / (T(1) - ar * cm - cr * ap);
            X[r] = rr * (X[r] - ar * xm - cr * xp);
            A[r] = -rr * ar * am;
            C[r] = -rr * cr * cp;
        }
        __syncthreads();
    }
    // row s - 1 is decoupled: X already holds its solution
    for (int t = s >> 1; t >= 1; t >>= 1) {
        const int cnt = (nz - (t - 1) + 2 * t - 1) / (2 * t);         // rows t-1 + 2t q < nz
        for (int w = tid; w < cnt * tp; w += kPcrThreads) {
            const int q = w / tp, pl = w - q * tp;
            const int z = t - 1 + 2 * t * q;
            const int r = z * tp + pl;
            const T um = (z - t >= 0) ? X[r - t * tp] : T(0);
            const T up = (z + t < nz) ? X[r + t * tp] : T(0);
            X[r] = X[r] - A[r] * um - C[r] * up;
        }
        __syncthreads();
    }
    tri_store<Tio>(S, a, base, m, b, p0, tp, X, red);
}

// Paired layout, for z lines up to 2048 (pcr_entries): both parts of TE entries
// per tile, per (z, entry) the complex right-hand side and the off-diagonals of
// the two parts (48 B), one thread per (z, entry) row working on both parts
// with 16- and 32-byte LDS accesses.  (Splitting every tile into single parts
// cost 30% at nz = 512: 6.0 -> 7.7 ms per PCR solve of 512^3.)
// Load TE z lines of slot m into LDS (rows r = z * TE + el), scaled and
// normalised to a unit diagonal; the zero mode pinned (row 0: u_0 = 0, row 1
// without its coupling to u_0).  X[r] = right-hand side, AC[r] = (a.x, a.y,
// c.x, c.y): lower and upper off-diagonals of the two parts.
template <typename Tio>
__device__ void tri_load2(const cplx<Tio>* __restrict__ S, const MidArgs<Tio>& a, size_t base, int m, int b, int e0,
                          int TE, cplx<double>* X, double* AC) {
    using T = double;
    const int nz = a.nz, ny = a.ny;
    const bool sing = a.singular && m == 0;
    const T proj = (sing && a.project) ? (T)(a.hz2 * a.mu[b]) : T(0);
    const T d0 = (a.bz0 == BC_D) ? T(-1) : T(1), d1 = (a.bz1 == BC_D) ? T(-1) : T(1);
    const int nrows = nz * TE;
    for (int r = threadIdx.x; r < nrows; r += kPcrThreads) {
        const int z = r / TE, el = r - z * TE, e = e0 + el;
        cplx<T> x = mk<T>(T(0), T(0));
        cplx<T> bm = mk<T>(T(1), T(1));
        if (e < ny) {
            const cplx<Tio> xs = S[base + (size_t)z * a.zstride + e];
            const cplx<Tio> bs = a.bmid[(size_t)m * ny + e];
            x = mk<T>((T)xs.x * (T)a.scale, (T)xs.y * (T)a.scale);
            bm = mk<T>((T)bs.x, (T)bs.y);
        }
        const bool pin = sing && e == 0;   // part x of the zero mode: row 0 reads u_0 = 0
        if (pin) x.x -= proj;
        cplx<T> bd = bm;
        if (z == 0) bd = mk<T>(bd.x + d0, bd.y + d0);
        if (z == nz - 1) bd = mk<T>(bd.x + d1, bd.y + d1);
        if (nz == 1) bd = mk<T>(bm.x + d0 + d1, bm.y + d0 + d1);
        const cplx<T> ib = mk<T>(T(1) / bd.x, T(1) / bd.y);
        T ax = (z > 0) ? ib.x : T(0), ay = (z > 0) ? ib.y : T(0);
        T cx = (z < nz - 1) ? ib.x : T(0), cy = (z < nz - 1) ? ib.y : T(0);
        T xx = x.x * ib.x, xy = x.y * ib.y;
        if (pin && z == 0) {
            ax = cx = T(0);
            xx = T(0);
        }
        if (pin && z == 1) ax = T(0);   // coupling to the pinned u_0 = 0
        X[r] = mk<T>(xx, xy);
        T* ac = AC + (size_t)r * 4;
        ac[0] = ax;
        ac[1] = ay;
        ac[2] = cx;
        ac[3] = cy;
    }
}

// Store the solved lines; the mean of the zero-mode line for the zero-mean gauge.
template <typename Tio>
__device__ void tri_store2(cplx<Tio>* __restrict__ S, const MidArgs<Tio>& a, size_t base, int m, int b, int e0,
                           int TE, const cplx<double>* X, double* red) {
    const int nz = a.nz, ny = a.ny;
    const bool sing = a.singular && m == 0;
    double csum = 0.0;
    for (int r = threadIdx.x; r < nz * TE; r += kPcrThreads) {
        const int z = r / TE, el = r - z * TE, e = e0 + el;
        if (e >= ny) continue;
        const cplx<double> u = X[r];
        S[base + (size_t)z * a.zstride + e] = mk<Tio>((Tio)u.x, (Tio)u.y);
        if (sing && e == 0) csum += u.x;
    }
    if (m == 0 && blockIdx.x == 0) {
        const double tot = block_sum<kPcrThreads>(csum, red);
        if (threadIdx.x == 0) a.cmean[b] = (sing && a.demean) ? tot / (double)nz : 0.0;
    }
}

template <typename Tio>
__global__ __launch_bounds__(kPcrThreads) void k_zpcr2(cplx<Tio>* __restrict__ S, MidArgs<Tio> a, int TE) {
    using T = double;
    constexpr int ITEMS = kPcrPairRows / kPcrThreads;   // (entry, z) rows per thread
    extern __shared__ __align__(16) unsigned char smem[];
    const int nz = a.nz;
    const int m = blockIdx.y, b = blockIdx.z;
    const int e0 = blockIdx.x * TE;
    const int tid = threadIdx.x;
    cplx<T>* X = reinterpret_cast<cplx<T>*>(smem);            // [z][TE]
    T* AC = reinterpret_cast<T*>(X + (size_t)nz * TE);         // [z][TE][4]: a.x, a.y, c.x, c.y
    double* red = reinterpret_cast<double*>(AC + (size_t)nz * TE * 4);
    const size_t base = (size_t)b * a.slots * nz * a.ny + (size_t)m * a.sstride;
    const int nrows = nz * TE;
    tri_load2<Tio>(S, a, base, m, b, e0, TE, X, AC);
    __syncthreads();
    for (int s = 1; s < nz; s <<= 1) {
        cplx<T> nx_[ITEMS];
        T na[ITEMS][4];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int r = tid + k * kPcrThreads;
            if (r >= nrows) continue;
            const int z = r / TE;
            const T* ac = AC + (size_t)r * 4;
            const cplx<T> x = X[r];
            T am[4] = {T(0), T(0), T(0), T(0)}, ap[4] = {T(0), T(0), T(0), T(0)};
            cplx<T> xm = mk<T>(T(0), T(0)), xp = xm;
            if (z - s >= 0) {
                const T* q = AC + (size_t)(r - s * TE) * 4;
                am[0] = q[0];
                am[1] = q[1];
                am[2] = q[2];
                am[3] = q[3];
                xm = X[r - s * TE];
            }
            if (z + s < nz) {
                const T* q = AC + (size_t)(r + s * TE) * 4;
                ap[0] = q[0];
                ap[1] = q[1];
                ap[2] = q[2];
                ap[3] = q[3];
                xp = X[r + s * TE];
            }
            // part x: a = ac[0], c = ac[2]; part y: a = ac[1], c = ac[3]
            const T rx = T(1) / (T(1) - ac[0] * am[2] - ac[2] * ap[0]);
            const T ry = T(1) / (T(1) - ac[1] * am[3] - ac[3] * ap[1]);
            na[k][0] = -rx * ac[0] * am[0];
            na[k][1] = -ry * ac[1] * am[1];
            na[k][2] = -rx * ac[2] * ap[2];
            na[k][3] = -ry * ac[3] * ap[3];
            nx_[k] = mk<T>(rx * (x.x - ac[0] * xm.x - ac[2] * xp.x), ry * (x.y - ac[1] * xm.y - ac[3] * xp.y));
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int r = tid + k * kPcrThreads;
            if (r >= nrows) continue;
            T* ac = AC + (size_t)r * 4;
            ac[0] = na[k][0];
            ac[1] = na[k][1];
            ac[2] = na[k][2];
            ac[3] = na[k][3];
            X[r] = nx_[k];
        }
        __syncthreads();
    }
    tri_store2<Tio>(S, a, base, m, b, e0, TE, X, red);
}

// Cyclic reduction with a parallel backward phase (section "Cyclic Reduction
// Technique", CR-P).  Forward: at stride s = 1, 2, 4, ... (while 2s <= nz) the
// rows z = 2s-1, 4s-1, ... are combined with rows z -+ s as in PCR,
//     r = 1 / (1 - a_z c_{z-s} - c_z a_{z+s})
//     a_z <- -r a_z a_{z-s},  c_z <- -r c_z c_{z+s},
//     x_z <- r (x_z - a_z x_{z-s} - c_z x_{z+s}),
// which leaves them coupled to rows z -+ 2s only; the rows a level reads are
// not the rows it writes, so a level needs one barrier.  The last stride s
// leaves the single row s-1, already decoupled (x = u).  Backward: for
// t = s/2, ..., 1 the rows z = t-1, 3t-1, ... take u_z = x_z - a_z u_{z-t} -
// c_z u_{z+t}, their neighbours being solved at the coarser levels.  Rows
// outside [0, nz) count as zero.
template <typename Tio>
__global__ __launch_bounds__(kPcrThreads) void k_zcr2(cplx<Tio>* __restrict__ S, MidArgs<Tio> a, int TE) {
    using T = double;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nz = a.nz;
    const int m = blockIdx.y, b = blockIdx.z;
    const int e0 = blockIdx.x * TE;
    const int tid = threadIdx.x;
    cplx<T>* X = reinterpret_cast<cplx<T>*>(smem);            // [z][TE]
    T* AC = reinterpret_cast<T*>(X + (size_t)nz * TE);         // [z][TE][4]: a.x, a.y, c.x, c.y
    double* red = reinterpret_cast<double*>(AC + (size_t)nz * TE * 4);
    const size_t base = (size_t)b * a.slots * nz * a.ny + (size_t)m * a.sstride;
    tri_load2<Tio>(S, a, base, m, b, e0, TE, X, AC);
    __syncthreads();
    int s = 1;
    for (; 2 * s <= nz; s <<= 1) {
        const int cnt = (nz - (2 * s - 1) + 2 * s - 1) / (2 * s);   // rows 2s-1 + 2s q < nz
        for (int w = tid; w < cnt * TE; w += kPcrThreads) {
            const int q = w / TE, el = w - q * TE;
            const int z = 2 * s - 1 + 2 * s * q;
            const int r = z * TE + el;
            T* ac = AC + (size_t)r * 4;
            const T* am = AC + (size_t)(r - s * TE) * 4;          // z - s >= s - 1 >= 0
            const cplx<T> xm = X[r - s * TE];
            T ap[4] = {T(0), T(0), T(0), T(0)};
            cplx<T> xp = mk<T>(T(0), T(0));
            if (z + s < nz) {
                const T* qq = AC + (size_t)(r + s * TE) * 4;
                ap[0] = qq[0];
                ap[1] = qq[1];
                ap[2] = qq[2];
                ap[3] = qq[3];
                xp = X[r + s * TE];
            }
            const cplx<T> x = X[r];
            const T rx = T(1) / (T(1) - ac[0] * am[2] - ac[2] * ap[0]);
            const T ry = T(1) / (T(1) - ac[1] * am[3] - ac[3] * ap[1]);
            const T a0 = -rx * ac[0] * am[0], a1 = -ry * ac[1] * am[1];
            const T c0 = -rx * ac[2] * ap[2], c1 = -ry * ac[3] * ap[3];
            X[r] = mk<T>(rx * (x.x - ac[0] * xm.x - ac[2] * xp.x), ry * (x.y - ac[1] * xm.y - ac[3] * xp.y));
            ac[0] = a0;
            ac[1] = a1;
            ac[2] = c0;
            ac[3] = c1;
        }
        __syncthreads();
    }
    // row s - 1 is decoupled: X already holds its solution
    for (int t = s >> 1; t >= 1; t >>= 1) {
        const int cnt = (nz - (t - 1) + 2 * t - 1) / (2 * t);         // rows t-1 + 2t q < nz
        for (int w = tid; w < cnt * TE; w += kPcrThreads) {
            const int q = w / TE, el = w - q * TE;
            const int z = t - 1 + 2 * t * q;
            const int r = z * TE + el;
            const T* ac = AC + (size_t)r * 4;
            cplx<T> um = mk<T>(T(0), T(0)), up = um;
            if (z - t >= 0) um = X[r - t * TE];
            if (z + t < nz) up = X[r + t * TE];
            const cplx<T> x = X[r];
            X[r] = mk<T>(x.x - ac[0] * um.x - ac[2] * up.x, x.y - ac[1] * um.y - ac[3] * up.y);
        }
        __syncthreads();
    }
    tri_store2<Tio>(S, a, base, m, b, e0, TE, X, red);
}

// y passes around a reduction kernel on whole z lines: cr = false for PCR,
// true for CR-P
template <typename T>
hipError_t launch_mid_pcr(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s, bool cr) {
    if (a.nz > kPcrRowsMax || a.ny > 512) return hipErrorInvalidValue;
    {
        // the largest tile any plan asks for, once per kernel and device
        const int maxb = (int)((size_t)kPcrRowsMax * 3 * sizeof(double) + 64 * sizeof(double));
        const int maxb2 = (int)((size_t)kPcrPairRows * (sizeof(double2) + 4 * sizeof(double)) + 64 * sizeof(double));
        const void* k1[2] = {reinterpret_cast<const void*>(k_zpcr<T>), reinterpret_cast<const void*>(k_zcr<T>)};
        const void* k2[2] = {reinterpret_cast<const void*>(k_zpcr2<T>), reinterpret_cast<const void*>(k_zcr2<T>)};
        for (int i = 0; i < 2; ++i) {
            hipError_t le = allow_dynamic_lds(k1[i], maxb);
            if (le == hipSuccess) le = allow_dynamic_lds(k2[i], maxb2);
            if (le != hipSuccess) return le;
        }
    }
    const dim3 gy(a.slots, (a.nz + 7) / 8, batch);
    hipLaunchKernelGGL((k_ypass<T, false>), gy, dim3(512), 0, s, S, a);
    const int te = pcr_entries(a.nz);
    if (te > 0) {
        const dim3 gz((a.ny + te - 1) / te, a.slots, batch);
        const size_t lds = pcr2_lds_bytes(a.nz);
        if (cr) hipLaunchKernelGGL((k_zcr2<T>), gz, dim3(kPcrThreads), lds, s, S, a, te);
        else hipLaunchKernelGGL((k_zpcr2<T>), gz, dim3(kPcrThreads), lds, s, S, a, te);
    } else {
        const int tp = pcr_parts(a.nz);
        const dim3 gz((2 * a.ny + tp - 1) / tp, a.slots, batch);
        const size_t lds = pcr_lds_bytes(a.nz);
        if (cr) hipLaunchKernelGGL((k_zcr<T>), gz, dim3(kPcrThreads), lds, s, S, a, tp);
        else hipLaunchKernelGGL((k_zpcr<T>), gz, dim3(kPcrThreads), lds, s, S, a, tp);
    }
    hipLaunchKernelGGL((k_ypass<T, true>), gy, dim3(512), 0, s, S, a);
    return hipGetLastError();
}

template hipError_t launch_mid_pcr<double>(cplx<double>*, const MidArgs<double>&, int, hipStream_t, bool);
template hipError_t launch_mid_pcr<float>(cplx<float>*, const MidArgs<float>&, int, hipStream_t, bool);

}  // namespace pp
