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

#include <type_traits>

#include "pp_kernels.hpp"

namespace pp {

// Per-lane share of a chunk: a wavefront owns planes wave, wave + NW, ...; its
// lanes hold elements y = lane + 64 k of each.  Register r of a lane covers
// plane p = r / epl and element k = r % epl of that plane (epl = ceil(ny/64)).
struct LaneSlot {
    int l, y;
};
__device__ __forceinline__ LaneSlot lane_slot(int r, int epl, float inv_epl, int wave, int nw, int lane) {
    const int p = fdiv(r, inv_epl);
    LaneSlot s;
    s.l = wave + nw * p;
    s.y = lane + 64 * (r - p * epl);
    return s;
}

// Planes whose pivots and right-hand sides are fetched ahead of each stretch of
// the (serial) z recurrences.
constexpr int kZBatch = 4;

// Tabulated reciprocal pivot of plane z for entry e (converged / last-row values come from registers).
template <typename T>
__device__ __forceinline__ cplx<T> row_pivot(const MidArgs<T>& a, int lmax, int roff, int z, int e, cplx<T> winf,
                                             cplx<T> wlast) {
    if (z == a.nz - 1) return wlast;
    if (z < lmax) return a.wrows[(size_t)(roff + z) * a.ny + e];
    return winf;
}

// The z march.  RMAX: chunk values per lane (64 * RMAX >= ny); OWN: y entries per
// thread in the z recurrences (NTH * OWN >= ny).
template <typename T, int NTH, int RMAX, int OWN>
__global__ __launch_bounds__(NTH) void k_zmarch(cplx<T>* __restrict__ S, MidArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NW = NTH / 64;
    const int m = blockIdx.x, b = blockIdx.y;
    const int ny = a.ny, nz = a.nz, ldy = a.ldy, zb = a.zb;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // LDS: zb planes of ny (padded), then the y twiddles
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* twl = lds + zb * ldy;
    for (int i = tid; i < ny; i += NTH) twl[i] = a.twy[i];
    cplx<T>* col = S + (size_t)b * a.slots * nz * ny + (size_t)m * a.sstride;
    const size_t zs = (size_t)a.zstride;
    const bool pairslot = (a.bx != BC_P) || (m == 0);
    const bool sep = (a.by == BC_P) && pairslot;
    const bool sing = a.singular && (m == 0);
    const int lmax = a.lmax[m], roff = a.rowoff[m];
    const T scale = a.scale;
    const T proj = (sing && a.project) ? (T)(a.hz2 * a.mu[b]) : T(0);
    const int half = (ny >> 1) + 1;
    const int nchunks = (nz + zb - 1) / zb;
    const int epl = (ny + 63) >> 6;
    const float inv_epl = 1.0f / (float)epl;
    const int ppw = (zb + NW - 1) / NW;          // planes per wave per chunk (ppw * epl <= RMAX)

    // owned z-recurrence entries e = tid + q * NTH; converged and last-row pivots in registers
    cplx<T> st[OWN], winf[OWN], wlast[OWN];
    // periodic z (Sherman-Morrison; see k_zpipe): y_0 accumulator, correction, q_{z+1}
    cplx<T> y0[OWN], corr[OWN], qn[OWN];
    const bool zper = a.zper != 0;
    const int alen = zper ? a.alen[m] : 0, aoff = zper ? a.aoff[m] : 0;
    const int qlen = zper ? a.qlen[m] : 0, qoff = zper ? a.qoff[m] : 0;
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
        const int e = tid + q * NTH;
        st[q] = mk<T>(T(0), T(0));
        winf[q] = st[q];
        wlast[q] = st[q];
        y0[q] = st[q];
        corr[q] = st[q];
        qn[q] = st[q];
        if (zper && e < ny) qn[q] = a.qlast[(size_t)m * ny + e];
        if (e < ny) {
            winf[q] = a.winf[(size_t)m * ny + e];
            wlast[q] = a.wlast[(size_t)m * ny + e];
        }
    }

    cplx<T> pre[RMAX];
    auto fetch = [&](int z0, int nl) {
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const LaneSlot ls = lane_slot(r, epl, inv_epl, wave, NW, lane);
            if (r < ppw * epl && ls.l < nl && ls.y < ny) pre[r] = col[(size_t)(z0 + ls.l) * zs + ls.y];
        }
    };

    // ------------------------------------------------------------- upward
    fetch(0, min(zb, nz));
    for (int c = 0; c < nchunks; ++c) {
        const int zc = c * zb;
        const int nl = min(zb, nz - zc);
        // own planes: prefetched values -> LDS, pre-processed for the y transform
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const LaneSlot ls = lane_slot(r, epl, inv_epl, wave, NW, lane);
            if (r < ppw * epl && ls.l < nl && ls.y < ny) {
                cplx<T> v = pre[r];
                int pos = ls.y;
                if (a.by != BC_P) {
                    pos = makhoul_pos(ls.y, ny);
                    if (a.by == BC_D && (ls.y & 1)) v = mk<T>(-v.x, -v.y);
                }
                lds[ls.l * ldy + pad(pos)] = v;
            }
        }
        if (c + 1 < nchunks) fetch(zc + zb, min(zb, nz - zc - zb));
        if (c == 0) __syncthreads();   // twiddles
        // forward y transform of each own plane, then its post-processing
        for (int l = wave; l < nl; l += NW) {
            cplx<T>* line = lds + l * ldy;
            wave_lds_sync();
            wfft<RMAX, false, T>(line, a.fy, twl, lane);
            if (a.by != BC_P) {
                // DCT-II post-twiddle over the pairs (k, ny-k)
                for (int k = lane; k < half; k += 64) {
                    if (k == 0) continue;
                    const cplx<T> vk = line[pad(k)];
                    const cplx<T> wk = a.mky[k];
                    if (2 * k == ny) {
                        line[pad(k)] = cscale(cadd(cmul(wk, vk), cmulc(vk, wk)), T(0.5));
                    } else {
                        const cplx<T> vr = line[pad(ny - k)];
                        const cplx<T> wr = a.mky[ny - k];
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
        }
        __syncthreads();
        // forward elimination across the chunk's planes, kZBatch planes at a time
        // (pivots and right-hand sides fetched ahead of the dependent steps);
        // eliminated right-hand sides go to HBM
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
                            w[j] = row_pivot(a, lmax, roff, zc + l, e, winf[q], wlast[q]);
                            d[j] = cscale(lds[l * ldy + pad(e)], scale);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < kZBatch; ++j) {
                        const int l = l0 + j;
                        if (l < nl) {
                            cplx<T> dd = d[j];
                            if (sing && e == 0) dd.x -= proj;
                            if (zper && zc + l < alen) {
                                const cplx<T> al = a.arows[(size_t)(aoff + zc + l) * ny + e];
                                y0[q].x += al.x * dd.x;
                                y0[q].y += al.y * dd.y;
                            }
                            prev = mk<T>((dd.x - prev.x) * w[j].x, (dd.y - prev.y) * w[j].y);
                            col[(size_t)(zc + l) * zs + e] = prev;
                        }
                    }
                }
                st[q] = prev;
            }
        }
        __syncthreads();
    }

    // ----------------------------------------------------------- downward
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
        const int e = tid + q * NTH;
        if (zper && e < ny) {
            // st is y_{n-1}, the last eliminated value
            const cplx<T> ig = a.inv_gamma[(size_t)m * ny + e], id = a.inv_den[(size_t)m * ny + e];
            corr[q] = mk<T>((y0[q].x + st[q].x * ig.x) * id.x, (y0[q].y + st[q].y * ig.y) * id.y);
        }
        st[q] = mk<T>(T(0), T(0));
    }
    double csum = 0.0;
    fetch((nchunks - 1) * zb, nz - (nchunks - 1) * zb);
    for (int c = nchunks - 1; c >= 0; --c) {
        const int zc = c * zb;
        const int nl = min(zb, nz - zc);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const LaneSlot ls = lane_slot(r, epl, inv_epl, wave, NW, lane);
            if (r < ppw * epl && ls.l < nl && ls.y < ny) lds[ls.l * ldy + pad(ls.y)] = pre[r];
        }
        if (c > 0) fetch(zc - zb, zb);
        __syncthreads();
        // back substitution across the chunk's planes, kZBatch planes at a time
#pragma unroll
        for (int q = 0; q < OWN; ++q) {
            const int e = tid + q * NTH;
            if (e < ny) {
                cplx<T> nxt = st[q];
                for (int l1 = nl - 1; l1 >= 0; l1 -= kZBatch) {
                    cplx<T> w[kZBatch], dp[kZBatch];
#pragma unroll
                    for (int j = 0; j < kZBatch; ++j) {
                        const int l = l1 - j;
                        if (l >= 0) {
                            w[j] = row_pivot(a, lmax, roff, zc + l, e, winf[q], wlast[q]);
                            dp[j] = lds[l * ldy + pad(e)];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < kZBatch; ++j) {
                        const int l = l1 - j;
                        if (l >= 0) {
                            nxt = mk<T>(dp[j].x - w[j].x * nxt.x, dp[j].y - w[j].y * nxt.y);
                            cplx<T> un = nxt;
                            if (zper) {
                                const int z = zc + l;
                                if (z != nz - 1) {
                                    const cplx<T> qp = (z < qlen) ? a.qrows[(size_t)(qoff + z) * ny + e]
                                                                  : mk<T>(T(0), T(0));
                                    qn[q] = mk<T>(qp.x - w[j].x * qn[q].x, qp.y - w[j].y * qn[q].y);
                                }
                                un = mk<T>(nxt.x - corr[q].x * qn[q].x, nxt.y - corr[q].y * qn[q].y);
                            }
                            lds[l * ldy + pad(e)] = un;
                            if (sing && e == 0) csum += (double)un.x;
                        }
                    }
                }
                st[q] = nxt;
            }
        }
        __syncthreads();
        // inverse y transform of each own plane, written straight to HBM
        for (int l = wave; l < nl; l += NW) {
            cplx<T>* line = lds + l * ldy;
            if (a.by != BC_P) {
                // DCT-III pre-twiddle: W_k = e^{+i pi k/2N} (X_k - i X_{N-k}), X_N = 0
                for (int k = lane; k < half; k += 64) {
                    if (k == 0) continue;
                    const cplx<T> xk = line[pad(k)];
                    if (2 * k == ny) {
                        line[pad(k)] = cmulc(mk<T>(xk.x + xk.y, xk.y - xk.x), a.mky[k]);
                    } else {
                        const cplx<T> xr = line[pad(ny - k)];
                        line[pad(k)] = cmulc(mk<T>(xk.x + xr.y, xk.y - xr.x), a.mky[k]);
                        line[pad(ny - k)] = cmulc(mk<T>(xr.x + xk.y, xr.y - xk.x), a.mky[ny - k]);
                    }
                }
            } else if (sep) {
                for (int k = lane; k < half; k += 64) {
                    if (k == 0 || 2 * k >= ny) continue;
                    const cplx<T> A = line[pad(k)], B = line[pad(ny - k)];
                    line[pad(k)] = mk<T>(A.x - B.y, A.y + B.x);        // A + i B
                    line[pad(ny - k)] = mk<T>(A.x + B.y, B.x - A.y);   // conj(A) + i conj(B)
                }
            }
            wave_lds_sync();
            wfft<RMAX, true, T>(line, a.fy, twl, lane);
            for (int y = lane; y < ny; y += 64) {
                int pos = y;
                if (a.by != BC_P) pos = makhoul_pos(y, ny);
                cplx<T> v = line[pad(pos)];
                if (a.by == BC_D && (y & 1)) v = mk<T>(-v.x, -v.y);
                col[(size_t)(zc + l) * zs + y] = v;
            }
        }
    }
    if (m == 0 && tid == 0) a.cmean[b] = (sing && a.demean) ? csum / (double)nz : 0.0;
}

// ---------------------------------------------------------------------------
// Pipelined z march for y lines of up to NYMAX = 512 (NW = 8 wavefronts), of
// exactly 384 (float, NW = 6) or of up to 1024 (float: NW = 8; double: NW = 4, so
// that a chunk of 1024-long double planes fits in LDS), and, segmented, of up
// to 256 (NW = 4, several workgroups per CU): the same stages as k_zmarch,
// arranged so that the memory traffic of one chunk overlaps the arithmetic of
// another.
//
// A chunk is NW planes, one per wavefront; a lane holds elements y = lane + 64 k
// of its wavefront's plane, and a thread owns the z recurrences of entries
// e = tid + 64 NW o (o < OWN = NYMAX / (64 NW)).  Upward, a lane prefetches its share of
// its wavefront's plane of the next chunk into registers while the current
// chunk is transformed and eliminated; the pivots of the next chunk are
// fetched after the current recurrences.  Downward, a thread prefetches its
// own entries of the 8 planes of the next chunk (the eliminated right-hand
// sides), so back substitution runs from registers, and each wavefront then
// transforms and stores one plane.
//
// The order of issue is chosen so that, with in-order completion of vector
// memory operations, every wait retires only what it needs: at each point of
// use, the operations issued after the awaited load are a fixed set (one
// chunk's stores, or one chunk's prefetch).  FULL (ny == NYMAX, the rows of
// the march a multiple of NW) removes every data-dependent branch around
// memory instructions, so the compiler can count them exactly; barriers order
// LDS only.  (The float halves of the split march load each chunk's pivots
// right before its recurrences instead: see LATEPIV.)
//
// Where the columns are few, the march of a column is split between two
// workgroups (PH 1 and 2 of zpipe_body, two launches): both halves eliminate
// toward a meeting point near the middle of z, then substitute away from it.
//
// The march itself is zpipe_body, which works in precision T on a column it
// reads (upward) from `icol` in precision Tin and writes (eliminated right-hand
// sides, and everything on the way down) to `ocol` in precision Tout; the
// plain solves run it in place (icol == ocol, one precision).  The refined
// solve's mixed march (k_zpipe_mixed) runs the slots of the smallest x
// wavenumbers in double from a double copy of their spectra and the others in
// float, both storing float.

// LDS of one march workgroup in compute precision T.
template <typename T, int NYMAX, int NW> struct ZpipeLds {
    static constexpr int LDY = NYMAX + NYMAX / 8;   // work-buffer plane stride (>= padded_len(NYMAX))
    cplx<T> work[NW * LDY];
    cplx<T> twl[NYMAX];
    cplx<T> mkl[NYMAX];
};

// Precisions: Tin of the column read upward, T of the z recurrences (and their
// tables, a), Tf of the y transforms (LDS lines, tables af), Tout of everything
// stored.  YFWD false: icol already holds the y-transformed values (k_ypre),
// so the way up only eliminates (each thread prefetches its own entries).
//
// PH 0: the whole march.  PH 1 and 2 split it between two workgroups per
// column (blockIdx.z = 0: rows 0 .. zsplit-1 from z = 0; 1: rows zsplit ..
// nz-1 from z = nz-1, through negated strides and the reversed system's
// pivots).  PH 1 eliminates toward the meeting rows and leaves each half's
// last eliminated value in zbuf; PH 2 solves the two meeting rows from them
// and substitutes away from the meeting point.  Both halves run the same code
// on their own rows, so the column has twice the workgroups in flight.
template <typename Tin, typename T, typename Tf, typename Tout, int NYMAX, int NW, bool FULL, bool PERZ, bool YFWD,
          int PH = 0>
__device__ __forceinline__ void zpipe_body(const cplx<Tin>* icol, ptrdiff_t izs, cplx<Tout>* ocol, ptrdiff_t zs,
                                           const MidArgs<T>& a, const MidArgs<Tf>& af,
                                           ZpipeLds<Tf, NYMAX, NW>& L) {
    constexpr int NTH = 64 * NW;
    constexpr int kSZ = NW;                      // planes per chunk = wavefronts per workgroup
    constexpr int EPL = NYMAX / 64;              // plane elements per lane
    constexpr int OWN = NYMAX / NTH;             // z-recurrence entries per thread
    constexpr int LDY = ZpipeLds<Tf, NYMAX, NW>::LDY;
    static_assert(EPL == kSZ * OWN, "one prefetch buffer serves both directions");
    cplx<Tf>* work = L.work;
    cplx<Tf>* twl = L.twl;
    cplx<Tf>* mkl = L.mkl;
    const int m = blockIdx.x, b = blockIdx.y;
    const int ny = FULL ? NYMAX : a.ny;
    static_assert(PH == 0 || !PERZ, "periodic z is one march");
    constexpr bool TWO = (PH == 1 || PH == 2);   // two-sided split
    constexpr bool SEG = (PH == 3 || PH == 4);   // segmented
    const int side = TWO ? (int)blockIdx.z : 0;
    const int seg = SEG ? (int)blockIdx.z : 0;
    const bool lastseg = SEG && seg == a.zsegs - 1;
    const bool fresh = SEG && seg > 0;            // pivots of a segment starting inside the column
    const int a0 = SEG ? seg * a.zseglen : 0;
    // rows of this march, in local order
    const int nz = SEG ? (lastseg ? a.nz - a0 : a.zseglen) : (TWO ? (side ? a.nz - a.zsplit : a.zsplit) : a.nz);
    if (side) {
        icol += (ptrdiff_t)(a.nz - 1) * izs;
        ocol += (ptrdiff_t)(a.nz - 1) * zs;
        izs = -izs;
        zs = -zs;
    }
    if (SEG) {
        icol += (ptrdiff_t)a0 * izs;
        ocol += (ptrdiff_t)a0 * zs;
    }
    const cplx<T>* wrows = side ? a.bwrows : (fresh ? a.fwrows : a.wrows);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int i = tid; i < ny; i += NTH) {
        twl[i] = af.twy[i];
        mkl[i] = af.mky[i];
    }
    // periodic y on lines of 512: the transforms take their first (forward) or
    // last (inverse) stage in registers (w512_*)
    constexpr bool R512 = FULL && NYMAX == 512;
    const bool reg512 = R512 && a.by == BC_P;
    // (float twiddles in registers in the whole march; the split march's
    // halves read them from LDS, to fit two workgroups per CU)
    constexpr bool TWREG = sizeof(Tf) == 4 && PH == 0;
    using Tw512 = std::conditional_t<TWREG, Tw512Reg<Tf>, Tw512Lds<Tf>>;
    Tw512 w512;
    if constexpr (TWREG) {
        if constexpr (R512) w512 = tw512_regs<Tf>(af.twy, lane);
    } else {
        w512 = Tw512Lds<Tf>{twl, lane};
    }
    const bool pairslot = (a.bx != BC_P) || (m == 0);
    const bool sep = (a.by == BC_P) && pairslot;
    const bool sing = a.singular && (m == 0);
    const int roff = side ? a.browoff[m] : (fresh ? a.frowoff[m] : a.rowoff[m]);
    const T scale = a.scale;
    const T proj = (sing && a.project) ? (T)(a.hz2 * a.mu[b]) : T(0);
    const int half = (ny >> 1) + 1;
    const int nchunks = (nz + kSZ - 1) / kSZ;
    const int last = (nchunks - 1) * kSZ;

    // this thread's z-recurrence entries (entries past ny read a valid dummy)
    int ec[OWN], elen[OWN];
    bool live[OWN];
    cplx<T> winf[OWN], wlast[OWN];
    // periodic z: y_0 accumulated on the way up, the correction c = (y_0 +
    // y_{n-1}/gamma)/den at the turn, and q_z rebuilt on the way down (the
    // Sherman-Morrison rows decay from z = 0, so only the first chunks read them)
    // (rows per entry: ael / qel; their maximum over the wavefront: alw / qlw,
    // so whole wavefronts skip the rows once their entries' values are zero)
    cplx<T> y0[OWN], corr[OWN], qnext[OWN];
    int aoff = 0, qoff = 0;
    int ael[OWN], qel[OWN], alw[OWN], qlw[OWN];
    if constexpr (PERZ) {
        aoff = a.aoff[m];
        qoff = a.qoff[m];
    }
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
        const int e = tid + NTH * o;
        live[o] = FULL || e < ny;
        ec[o] = live[o] ? e : 0;
        winf[o] = (side ? a.bwinf : (fresh ? a.fwinf : a.winf))[(size_t)m * ny + ec[o]];
        elen[o] = (side ? a.belen : (fresh ? a.felen : a.elen))[(size_t)m * ny + ec[o]];
        wlast[o] = (lastseg ? a.flast : a.wlast)[(size_t)m * ny + ec[o]];
        y0[o] = mk<T>(T(0), T(0));
        corr[o] = y0[o];
        qnext[o] = y0[o];
        if constexpr (PERZ) {
            qnext[o] = a.qlast[(size_t)m * ny + ec[o]];
            ael[o] = live[o] ? a.aelen[(size_t)m * ny + ec[o]] : 0;
            qel[o] = live[o] ? a.qelen[(size_t)m * ny + ec[o]] : 0;
            int x = ael[o], y = qel[o];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                x = max(x, __shfl_xor(x, off, 64));
                y = max(y, __shfl_xor(y, off, 64));
            }
            alw[o] = __builtin_amdgcn_readfirstlane(x);
            qlw[o] = __builtin_amdgcn_readfirstlane(y);
        }
    }

    // reciprocal pivots of planes zc .. zc+NW-1 for the thread's entries (planes
    // past the entry's own rows read the first table element, which always
    // exists; the value then comes from winf / wlast); plane l, entry o at
    // l * OWN + o
    cplx<T> pv[kSZ * OWN];
    auto load_piv = [&](int zc) __attribute__((always_inline)) {
#pragma unroll
        for (int l = 0; l < kSZ; ++l) {
            const int z = zc + l;
#pragma unroll
            for (int o = 0; o < OWN; ++o) {
                // lanes past their entry's rows read the same element (one cache line)
                const cplx<T>* src = (z < elen[o]) ? wrows + (size_t)(roff + z) * ny + ec[o] : wrows;
                pv[l * OWN + o] = *src;
            }
        }
    };
    // (component-wise selects between values, so that the arrays stay in registers)
    auto pivot = [&](int z, int l, int o) __attribute__((always_inline)) -> cplx<T> {
        const cplx<T> p = pv[l * OWN + o], wi = winf[o], wl = wlast[o];
        const bool lastrow = (PH == 0 || lastseg) && (z == nz - 1), tab = (z < elen[o]);
        return mk<T>(lastrow ? wl.x : (tab ? p.x : wi.x), lastrow ? wl.y : (tab ? p.y : wi.y));
    };
    // upward prefetch (clamped to the last plane): YFWD, elements y = lane + 64 k
    // of plane zc + wave; otherwise the thread's own entries of planes zc .. zc+NW-1
    cplx<T> pre[EPL];
    auto load_plane = [&](int zc) __attribute__((always_inline)) {
        if constexpr (YFWD) {
            const cplx<Tin>* src = icol + (ptrdiff_t)min(zc + wave, nz - 1) * izs;
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                const int y = lane + 64 * k;
                pre[k] = cvt<T>(src[(FULL || y < ny) ? y : 0]);
            }
        } else {
#pragma unroll
            for (int l = 0; l < kSZ; ++l) {
#pragma unroll
                for (int o = 0; o < OWN; ++o)
                    pre[l * OWN + o] = cvt<T>(icol[(ptrdiff_t)min(zc + l, nz - 1) * izs + ec[o]]);
            }
        }
    };
    // downward prefetch: the thread's entries of planes zc .. zc+NW-1 (clamped to the last plane)
    auto load_entry = [&](int zc) __attribute__((always_inline)) {
#pragma unroll
        for (int l = 0; l < kSZ; ++l) {
#pragma unroll
            for (int o = 0; o < OWN; ++o) pre[l * OWN + o] = cvt<T>(ocol[(ptrdiff_t)min(zc + l, nz - 1) * zs + ec[o]]);
        }
    };

    // ------------------------------------------------------------- upward
    cplx<T> st[OWN];
    // segmented march: the segment's local solution at its first row,
    // sum_z tau_z y_z with tau the back substitution's running product
    cplx<T> ga[PH == 3 ? OWN : 1], tau[PH == 3 ? OWN : 1];
#pragma unroll
    for (int o = 0; o < OWN; ++o) st[o] = mk<T>(T(0), T(0));
    if constexpr (PH == 3) {
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            ga[o] = mk<T>(T(0), T(0));
            tau[o] = mk<T>(T(1), T(1));
        }
    }
    // the split march's float halves load each chunk's pivots just before its
    // recurrences (registers: their prefetch would be live across the transforms)
    constexpr bool LATEPIV = PH != 0 && sizeof(Tf) == 4 && sizeof(T) == 4;
    if constexpr (PH != 2 && PH != 4) {
        load_plane(0);
        if constexpr (!LATEPIV) load_piv(0);
    }
    auto up_chunk = [&](int c) __attribute__((always_inline)) {
        const int zc = c * kSZ;
        const int nl = FULL ? kSZ : min(kSZ, nz - zc);
        // !YFWD: this chunk's right-hand sides, taken out of the prefetch buffer
        cplx<T> cur[YFWD ? 1 : EPL];
        if constexpr (!YFWD) {
#pragma unroll
            for (int k = 0; k < EPL; ++k) cur[k] = pre[k];
            load_plane(min(zc + kSZ, last));
        } else {
        lds_barrier();   // the previous recurrences are done with the work buffer
        cplx<Tf>* line = work + wave * LDY;
        const bool own = FULL || wave < nl;
        cplx<Tf> v[EPL];
        if (reg512) {
#pragma unroll
            for (int k = 0; k < EPL; ++k) v[k] = cvt<Tf>(pre[k]);
        } else if (own) {
            // prefetched plane -> work plane, reordered for the forward transform
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                const int y = lane + 64 * k;
                if (FULL || y < ny) {
                    cplx<Tf> x = cvt<Tf>(pre[k]);
                    int pos = y;
                    if (a.by != BC_P) {
                        pos = makhoul_pos(y, ny);
                        if (a.by == BC_D && (y & 1)) x = mk<Tf>(-x.x, -x.y);
                    }
                    line[pad(pos)] = x;
                }
            }
        }
        load_plane(min(zc + kSZ, last));
        if (reg512) {
            if constexpr (R512) {
                w512_first<false, Tf>(v, line, lane);
                w512_second<false, Tf>(line, w512, lane);
                w512_last<false, Tf>(line, w512, lane, v);
            }
            // each lane writes back the elements it read
#pragma unroll
            for (int t = 0; t < EPL; ++t) line[pad(lane + 64 * t)] = v[t];
            if (sep) {
                wave_lds_sync();
                for (int k = lane; k < half; k += 64) {
                    if (k == 0 || 2 * k >= ny) continue;
                    const cplx<Tf> zk = line[pad(k)], zr = line[pad(ny - k)];
                    line[pad(k)] = mk<Tf>(Tf(0.5) * (zk.x + zr.x), Tf(0.5) * (zk.y - zr.y));
                    line[pad(ny - k)] = mk<Tf>(Tf(0.5) * (zk.y + zr.y), Tf(0.5) * (zr.x - zk.x));
                }
            }
        } else if (own) {
            wave_lds_sync();
            wfft<EPL, false, Tf>(line, af.fy, twl, lane);
            if (a.by != BC_P) {
                for (int k = lane; k < half; k += 64) {
                    if (k == 0) continue;
                    const cplx<Tf> vk = line[pad(k)];
                    const cplx<Tf> wk = mkl[k];
                    if (2 * k == ny) {
                        line[pad(k)] = cscale(cadd(cmul(wk, vk), cmulc(vk, wk)), Tf(0.5));
                    } else {
                        const cplx<Tf> vr = line[pad(ny - k)];
                        const cplx<Tf> wr = mkl[ny - k];
                        line[pad(k)] = cscale(cadd(cmul(wk, vk), cmulc(vr, wk)), Tf(0.5));
                        line[pad(ny - k)] = cscale(cadd(cmul(wr, vr), cmulc(vk, wr)), Tf(0.5));
                    }
                }
            } else if (sep) {
                for (int k = lane; k < half; k += 64) {
                    if (k == 0 || 2 * k >= ny) continue;
                    const cplx<Tf> zk = line[pad(k)], zr = line[pad(ny - k)];
                    line[pad(k)] = mk<Tf>(Tf(0.5) * (zk.x + zr.x), Tf(0.5) * (zk.y - zr.y));
                    line[pad(ny - k)] = mk<Tf>(Tf(0.5) * (zk.y + zr.y), Tf(0.5) * (zr.x - zk.x));
                }
            }
        }
        lds_barrier();
        }
        if constexpr (LATEPIV) load_piv(zc);
        // forward elimination over the chunk; eliminated right-hand sides go to HBM
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            if (!live[o]) continue;
            const int e = ec[o];
            cplx<T> al[PERZ ? kSZ : 1];
            if constexpr (PERZ) {
                if (zc < alw[o]) {
#pragma unroll
                    for (int l = 0; l < kSZ; ++l)
                        al[l] = (zc + l < ael[o]) ? a.arows[(size_t)(aoff + zc + l) * ny + e] : mk<T>(T(0), T(0));
                }
            }
            cplx<T> prev = st[o];
#pragma unroll
            for (int l = 0; l < kSZ; ++l) {
                if (FULL || l < nl) {
                    const int z = zc + l;
                    const cplx<T> w = pivot(z, l, o);
                    cplx<T> d;
                    if constexpr (YFWD) d = cscale(cvt<T>(work[l * LDY + pad(e)]), scale);
                    else d = cscale(cur[l * OWN + o], scale);
                    if (sing && e == 0) d.x -= proj;
                    if constexpr (PERZ) {
                        if (zc < alw[o]) {
                            y0[o].x += al[l].x * d.x;
                            y0[o].y += al[l].y * d.y;
                        }
                    }
                    prev = mk<T>((d.x - prev.x) * w.x, (d.y - prev.y) * w.y);
                    ocol[(ptrdiff_t)z * zs + e] = cvt<Tout>(prev);
                    if constexpr (PH == 3) {
                        ga[o] = mk<T>(ga[o].x + tau[o].x * prev.x, ga[o].y + tau[o].y * prev.y);
                        tau[o] = mk<T>(-w.x * tau[o].x, -w.y * tau[o].y);
                    }
                }
            }
            st[o] = prev;
        }
        if constexpr (!LATEPIV) load_piv(min(zc + kSZ, last));   // the last chunk reloads its own pivots for the way down
    };
    // the first chunk is issued outside the loop so that every pass through the
    // loop sees the same sequence of memory operations before it
    if constexpr (PH != 2 && PH != 4) {
        up_chunk(0);
        for (int c = 1; c < nchunks; ++c) up_chunk(c);
    }
    if constexpr (PH == 1) {
        // this half's last eliminated values, for the meeting rows
#pragma unroll
        for (int o = 0; o < OWN; ++o)
            if (live[o]) a.zbuf[(((size_t)b * a.slots + m) * 2 + side) * ny + ec[o]] = st[o];
        if (side == 0 && m == 0 && tid == 0) a.cmean[b] = 0.0;   // the halves add their shares in PH 2
        return;
    }
    if constexpr (PH == 3) {
        // the segment's local solution at its first and last rows (the last
        // is the last eliminated value), for the reduced system
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            if (!live[o]) continue;
            cplx<T>* g = a.segg + (((size_t)b * a.slots + m) * a.zsegs + seg) * 2 * ny + ec[o];
            g[0] = ga[o];
            g[ny] = st[o];
        }
        if (seg == 0 && m == 0 && tid == 0) a.cmean[b] = 0.0;   // the segments add their shares in PH 4
        return;
    }

    // ----------------------------------------------------------- downward
    // the top chunk's eliminated right-hand sides were stored by this thread
    // (same entries, same addresses): read them back in program order
    if constexpr ((PH == 2 || PH == 4) && !LATEPIV) load_piv(last);
    load_entry(last);
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
        if constexpr (PERZ) {
            // st is y_{n-1}, the last eliminated value
            const cplx<T> ig = a.inv_gamma[(size_t)m * ny + ec[o]], id = a.inv_den[(size_t)m * ny + ec[o]];
            corr[o] = mk<T>((y0[o].x + st[o].x * ig.x) * id.x, (y0[o].y + st[o].y * ig.y) * id.y);
        }
        if constexpr (PH == 2) {
            // the meeting rows k-1 and k from the halves' last eliminated values
            // (upper yu = y_{k-1}, lower yl = y'_k): u_{k-1} = yu - w u_k and
            // u_k = yl - v u_{k-1}; each half starts from its neighbour across
            // the meeting point, g = 1 / (1 - v w)
            const size_t zb = ((size_t)b * a.slots + m) * 2 * ny + ec[o];
            const cplx<T> yu = a.zbuf[zb], yl = a.zbuf[zb + ny];
            const cplx<T>* mt = a.meet + ((size_t)m * ny + ec[o]) * 3;
            const cplx<T> w = mt[0], v = mt[1], g = mt[2];
            st[o] = side ? mk<T>(g.x * (yu.x - w.x * yl.x), g.y * (yu.y - w.y * yl.y))
                         : mk<T>(g.x * (yl.x - v.x * yu.x), g.y * (yl.y - v.y * yu.y));
        } else {
            st[o] = mk<T>(T(0), T(0));
        }
    }
    // segmented march: the couplings above (cl) and below (cr) this segment,
    // and the rows of rho (per entry: rel, wavefront maximum: rlw)
    cplx<T> cl[PH == 4 ? OWN : 1], cr[PH == 4 ? OWN : 1], rhol[PH == 4 ? OWN : 1];
    int rel[PH == 4 ? OWN : 1], rlw[PH == 4 ? OWN : 1];
    int rroff = 0;
    if constexpr (PH == 4) {
        rroff = fresh ? a.rrowoff[m] : 0;
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            const cplx<T>* lr = a.seglr + (((size_t)b * a.slots + m) * a.zsegs + seg) * 2 * ny + ec[o];
            cl[o] = lr[0];
            cr[o] = lr[ny];
            rhol[o] = a.rholast[(size_t)m * ny + ec[o]];
            rel[o] = (fresh && live[o]) ? a.relen[(size_t)m * ny + ec[o]] : 0;
            int x = rel[o];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
            rlw[o] = __builtin_amdgcn_readfirstlane(x);
        }
    }
    double csum = 0.0;
    auto down_chunk = [&](int c) __attribute__((always_inline)) {
        const int zc = c * kSZ;
        const int nl = FULL ? kSZ : min(kSZ, nz - zc);
        lds_barrier();   // the previous inverse transforms are done with the work buffer
        if constexpr (LATEPIV) load_piv(zc);
        // back substitution over the chunk, from registers into the work buffer
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            if (!live[o]) continue;
            const int e = ec[o];
            cplx<T> qv[PERZ ? kSZ : 1];
            if constexpr (PERZ) {
                if (zc < qlw[o]) {
#pragma unroll
                    for (int l = 0; l < kSZ; ++l)
                        qv[l] = (zc + l < qel[o]) ? a.qrows[(size_t)(qoff + zc + l) * ny + e] : mk<T>(T(0), T(0));
                }
            }
            cplx<T> rv[PH == 4 ? kSZ : 1];
            if constexpr (PH == 4) {
                if (zc < rlw[o]) {
#pragma unroll
                    for (int l = 0; l < kSZ; ++l)
                        rv[l] = (zc + l < rel[o]) ? a.rrows[(size_t)(rroff + zc + l) * ny + e] : mk<T>(T(0), T(0));
                }
            }
            cplx<T> nxt = st[o];
#pragma unroll
            for (int j = 0; j < kSZ; ++j) {
                const int l = kSZ - 1 - j;
                if (FULL || l < nl) {
                    const int z = zc + l;
                    const cplx<T> w = pivot(z, l, o);
                    cplx<T> dp = pre[l * OWN + o];
                    if constexpr (PH == 4) {
                        // the couplings moved to the right-hand side: the row
                        // above the segment through rho, the row below it at the
                        // segment's last row through that row's pivot
                        if (fresh) {
                            cplx<T> r = (zc < rlw[o]) ? rv[l] : mk<T>(T(0), T(0));
                            if (lastseg && z == nz - 1) r = rhol[o];
                            dp = mk<T>(dp.x - cl[o].x * r.x, dp.y - cl[o].y * r.y);
                        }
                        if (!lastseg && z == nz - 1) dp = mk<T>(dp.x - cr[o].x * w.x, dp.y - cr[o].y * w.y);
                    }
                    nxt = mk<T>(dp.x - w.x * nxt.x, dp.y - w.y * nxt.y);
                    cplx<T> un = nxt;
                    if constexpr (PERZ) {
                        // q_z of the rank-one vector, then u_z = y_z - c q_z
                        if (z != nz - 1) {
                            const cplx<T> qp = (zc < qlw[o]) ? qv[l] : mk<T>(T(0), T(0));
                            qnext[o] = mk<T>(qp.x - w.x * qnext[o].x, qp.y - w.y * qnext[o].y);
                        }
                        un = mk<T>(nxt.x - corr[o].x * qnext[o].x, nxt.y - corr[o].y * qnext[o].y);
                    }
                    work[l * LDY + pad(e)] = cvt<Tf>(un);
                    if (sing && e == 0) csum += (double)un.x;
                }
            }
            st[o] = nxt;
        }
        lds_barrier();
        const int zn = zc >= kSZ ? zc - kSZ : 0;
        load_entry(zn);
        if constexpr (!LATEPIV) load_piv(zn);
        // inverse y transform of this wave's plane, written straight to HBM
        if (FULL || wave < nl) {
            cplx<Tf>* line = work + wave * LDY;
            if (a.by != BC_P) {
                for (int k = lane; k < half; k += 64) {
                    if (k == 0) continue;
                    const cplx<Tf> xk = line[pad(k)];
                    if (2 * k == ny) {
                        line[pad(k)] = cmulc(mk<Tf>(xk.x + xk.y, xk.y - xk.x), mkl[k]);
                    } else {
                        const cplx<Tf> xr = line[pad(ny - k)];
                        line[pad(k)] = cmulc(mk<Tf>(xk.x + xr.y, xk.y - xr.x), mkl[k]);
                        line[pad(ny - k)] = cmulc(mk<Tf>(xr.x + xk.y, xr.y - xk.x), mkl[ny - k]);
                    }
                }
            } else if (sep) {
                for (int k = lane; k < half; k += 64) {
                    if (k == 0 || 2 * k >= ny) continue;
                    const cplx<Tf> A = line[pad(k)], B = line[pad(ny - k)];
                    line[pad(k)] = mk<Tf>(A.x - B.y, A.y + B.x);
                    line[pad(ny - k)] = mk<Tf>(A.x + B.y, B.x - A.y);
                }
            }
            wave_lds_sync();
            cplx<Tout>* dst = ocol + (ptrdiff_t)(zc + wave) * zs;
            if (reg512) {
                cplx<Tf> v[EPL];
                if constexpr (R512) {
                    w512_first_lds<true, Tf>(line, lane);
                    w512_second<true, Tf>(line, w512, lane);
                    w512_last<true, Tf>(line, w512, lane, v);
                }
#pragma unroll
                for (int t = 0; t < EPL; ++t) dst[lane + 64 * t] = cvt<Tout>(v[t]);
            } else {
                wfft<EPL, true, Tf>(line, af.fy, twl, lane);
#pragma unroll
                for (int k = 0; k < EPL; ++k) {
                    const int y = lane + 64 * k;
                    if (FULL || y < ny) {
                        int pos = y;
                        if (a.by != BC_P) pos = makhoul_pos(y, ny);
                        cplx<Tf> x = line[pad(pos)];
                        if (a.by == BC_D && (y & 1)) x = mk<Tf>(-x.x, -x.y);
                        dst[y] = cvt<Tout>(x);
                    }
                }
            }
        }
    };
    down_chunk(nchunks - 1);
    for (int c = nchunks - 2; c >= 0; --c) down_chunk(c);
    if constexpr (PH == 2 || PH == 4) {
        if (m == 0 && tid == 0 && sing && a.demean) atomicAdd(&a.cmean[b], csum / (double)a.nz);
    } else {
        if (m == 0 && tid == 0) a.cmean[b] = (sing && a.demean) ? csum / (double)nz : 0.0;
    }
}

// Waves per SIMD a march kernel is compiled for: the split march's halves in
// float on lines up to 512 at 4 (at most 128 VGPRs: two 512-thread
// workgroups per CU; 512^3 float march 0.51 -> 0.46 ms); the segmented
// four-wavefront march of lines up to 256 at 4 in float and 3 in double (no
// spills; 256^3 with 128 columns: float 0.143 -> 0.100 ms, double 0.182 ->
// 0.171 ms against the split march); everything else at 1 (the registers it
// needs).
template <typename T, int NYMAX, int PH> constexpr int zpipe_min_waves() {
    if (NYMAX == 256) return sizeof(T) == 4 ? 4 : 3;
    return (PH != 0 && sizeof(T) == 4 && NYMAX <= 512) ? 4 : 1;
}

// The march in one precision, in place.
template <typename T, int NYMAX, int NW, bool FULL, bool PERZ, int PH>
__global__ __launch_bounds__(64 * NW, (zpipe_min_waves<T, NYMAX, PH>())) void k_zpipe(cplx<T>* __restrict__ S, MidArgs<T> a) {
    __shared__ __align__(16) ZpipeLds<T, NYMAX, NW> L;
    cplx<T>* col = S + (size_t)blockIdx.y * a.slots * a.nz * a.ny + (size_t)blockIdx.x * a.sstride;
    zpipe_body<T, T, T, T, NYMAX, NW, FULL, PERZ, true, PH>(col, a.zstride, col, a.zstride, a, a, L);
}

// The refined solve's march: slots lo0 .. lo0+nlo-1 (the smallest x
// wavenumbers, whose z systems are the least well conditioned) take their
// right-hand sides from Slo[b][z][k][y], already transformed along y in double
// (k_ypre), and run the recurrences in double; everything else is float, and
// every result goes to S in float.  One workgroup per slot as in k_zpipe; the
// branch is uniform over the workgroup.  (Doing the double slots' y transforms
// here instead made those workgroups the last to finish: 0.69 against 0.52 ms
// at 512^3.)
// (lines of 384 only: on lines of 512 the double slots' registers spill at 4)
template <int NYMAX, int NW, bool FULL, bool PERZ, int PH>
__global__ __launch_bounds__(64 * NW, (zpipe_min_waves<float, NYMAX == 384 ? 384 : 1024, PH>())) void k_zpipe_mixed(const cplx<double>* __restrict__ Slo,
                                                         cplx<float>* __restrict__ S, MidArgs<double> ad,
                                                         MidArgs<float> af, int lo0, int nlo) {
    __shared__ __align__(16) ZpipeLds<float, NYMAX, NW> L;
    const int k = (int)blockIdx.x - lo0;
    cplx<float>* col = S + (size_t)blockIdx.y * af.slots * af.nz * af.ny + (size_t)blockIdx.x * af.sstride;
    if (k >= 0 && k < nlo) {
        const cplx<double>* icol = Slo + ((size_t)blockIdx.y * af.nz * nlo + k) * af.ny;
        zpipe_body<double, double, float, float, NYMAX, NW, FULL, PERZ, false, PH>(icol, (ptrdiff_t)nlo * af.ny, col,
                                                                                   af.zstride, ad, af, L);
    } else {
        zpipe_body<float, float, float, float, NYMAX, NW, FULL, PERZ, true, PH>(col, af.zstride, col, af.zstride, af,
                                                                                af, L);
    }
}

// Forward y transform, in double and in place, of the double slots of the
// refined solve (Slo[b][z][k][y], k < nlo, slot lo0 + k): one wavefront per
// plane, four planes per workgroup; the same pre- and post-processing as the
// march's upward transform.
constexpr int kYpreWaves = 4;
template <int EPL>
__global__ __launch_bounds__(64 * kYpreWaves) void k_ypre(cplx<double>* __restrict__ Slo, MidArgs<double> a,
                                                           int lo0, int nlo, int nplanes) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int ny = a.ny, ldy = a.ldy;
    cplx<double>* twl = reinterpret_cast<cplx<double>*>(smem);
    cplx<double>* mkl = twl + ny;
    cplx<double>* line = mkl + ny + (threadIdx.x >> 6) * ldy;
    for (int i = threadIdx.x; i < ny; i += 64 * kYpreWaves) {
        twl[i] = a.twy[i];
        mkl[i] = a.mky[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int pl = blockIdx.x * kYpreWaves + (threadIdx.x >> 6);   // plane index (b, z, k)
    if (pl >= nplanes) return;
    const int k = pl % nlo;
    const int m = lo0 + k;
    const bool pairslot = (a.bx != BC_P) || (m == 0);
    const bool sep = (a.by == BC_P) && pairslot;
    const int half = (ny >> 1) + 1;
    cplx<double>* src = Slo + (size_t)pl * ny;
    for (int y = lane; y < ny; y += 64) {
        cplx<double> x = src[y];
        int pos = y;
        if (a.by != BC_P) {
            pos = makhoul_pos(y, ny);
            if (a.by == BC_D && (y & 1)) x = mk<double>(-x.x, -x.y);
        }
        line[pad(pos)] = x;
    }
    wave_lds_sync();
    wfft<EPL, false, double>(line, a.fy, twl, lane);
    if (a.by != BC_P) {
        for (int q = lane; q < half; q += 64) {
            if (q == 0) continue;
            const cplx<double> vk = line[pad(q)];
            const cplx<double> wk = mkl[q];
            if (2 * q == ny) {
                line[pad(q)] = cscale(cadd(cmul(wk, vk), cmulc(vk, wk)), 0.5);
            } else {
                const cplx<double> vr = line[pad(ny - q)];
                const cplx<double> wr = mkl[ny - q];
                line[pad(q)] = cscale(cadd(cmul(wk, vk), cmulc(vr, wk)), 0.5);
                line[pad(ny - q)] = cscale(cadd(cmul(wr, vr), cmulc(vk, wr)), 0.5);
            }
        }
    } else if (sep) {
        for (int q = lane; q < half; q += 64) {
            if (q == 0 || 2 * q >= ny) continue;
            const cplx<double> zk = line[pad(q)], zr = line[pad(ny - q)];
            line[pad(q)] = mk<double>(0.5 * (zk.x + zr.x), 0.5 * (zk.y - zr.y));
            line[pad(ny - q)] = mk<double>(0.5 * (zk.y + zr.y), 0.5 * (zr.x - zk.x));
        }
    }
    wave_lds_sync();
    for (int y = lane; y < ny; y += 64) src[y] = line[pad(y)];
}

// Every chunk of the march (of both halves, or of every segment) whole.
template <typename T> static bool pipe_full(const MidArgs<T>& a, int nymax, int nw) {
    if (a.ny != nymax) return false;
    if (a.zsegs > 0) return a.zseglen % nw == 0 && (a.nz - (a.zsegs - 1) * a.zseglen) % nw == 0;
    if (a.zsplit > 0) return a.zsplit % nw == 0 && (a.nz - a.zsplit) % nw == 0;
    return a.nz % nw == 0;
}

// Segmented march, between its two launches: per (batch entry, slot, entry)
// one thread solves the reduced system of the segments' end rows.  Segment t's
// first and last values are X_t = Ga_t - L_t pa_t - R_t qa_t and Z_t = Gb_t -
// L_t pb_t - R_t qb_t (G the segment's local solution, L_t = Z_{t-1} the row
// above it, R_t = X_{t+1} the row below, p / q the responses to those rows);
// eliminated forward as Z_t = al_t + be_t X_{t+1}, X_t = ga_t + de_t X_{t+1},
// then solved backward from X_{P-1} = ga_{P-1}.  Each part (real system) on
// its own.  The forward coefficients stay in registers (loops unrolled over
// the largest segment count, guarded by the plan's), and the launch has
// workgroups of one wavefront, so that every CU takes a share.
template <typename T> __global__ __launch_bounds__(64) void k_zseg_reduce(MidArgs<T> a, int batch) {
    constexpr int PM = kMaxZSegments;
    const size_t i = (size_t)blockIdx.x * 64 + threadIdx.x;
    const int ny = a.ny, P = a.zsegs;
    if (i >= (size_t)batch * a.slots * ny) return;
    const int e = (int)(i % ny);
    const size_t bm = i / ny;
    const int m = (int)(bm % a.slots);
    const cplx<T>* K = a.segk + ((size_t)m * ny + e) * 12;
    const cplx<T>* G = a.segg + bm * P * 2 * ny + e;
    cplx<T>* LR = a.seglr + bm * P * 2 * ny + e;
    auto kk = [&](int t, int j) { return K[(t == 0 ? 0 : (t == P - 1 ? 8 : 4)) + j]; };
    auto mul = [](cplx<T> x, cplx<T> y) { return mk<T>(x.x * y.x, x.y * y.y); };
    auto sub = [](cplx<T> x, cplx<T> y) { return mk<T>(x.x - y.x, x.y - y.y); };
    auto add = [](cplx<T> x, cplx<T> y) { return mk<T>(x.x + y.x, x.y + y.y); };
    cplx<T> wal[PM], wbe[PM], wga[PM], wde[PM];
    cplx<T> al = G[ny];
    cplx<T> be = mk<T>(-kk(0, 3).x, -kk(0, 3).y);
    wal[0] = al;
    wbe[0] = be;
    cplx<T> ga = al;
#pragma unroll
    for (int t = 1; t < PM; ++t) {
        wal[t] = wbe[t] = wga[t] = wde[t] = mk<T>(T(0), T(0));
        if (t < P) {
            const cplx<T> pa = kk(t, 0), pb = kk(t, 1), qa = kk(t, 2), qb = kk(t, 3);
            const cplx<T> den = add(mk<T>(T(1), T(1)), mul(pa, be));
            const cplx<T> num = sub(G[(size_t)t * 2 * ny], mul(pa, al));
            ga = mk<T>(num.x / den.x, num.y / den.y);
            const cplx<T> de = mk<T>(-qa.x / den.x, -qa.y / den.y);
            wga[t] = ga;
            wde[t] = de;
            if (t < P - 1) {
                al = sub(G[((size_t)t * 2 + 1) * ny], mul(pb, add(al, mul(be, ga))));
                const cplx<T> nb = add(mul(mul(pb, be), de), qb);
                be = mk<T>(-nb.x, -nb.y);
                wal[t] = al;
                wbe[t] = be;
            }
        }
    }
    cplx<T> X = ga;   // X_{P-1}
    LR[0] = mk<T>(T(0), T(0));                          // nothing above segment 0
    LR[((size_t)(P - 1) * 2 + 1) * ny] = mk<T>(T(0), T(0));   // nothing below the last
#pragma unroll
    for (int t = PM - 2; t >= 0; --t) {
        if (t <= P - 2) {
            const cplx<T> Z = add(wal[t], mul(wbe[t], X));
            LR[((size_t)(t + 1) * 2) * ny] = Z;          // the row above segment t+1
            LR[((size_t)t * 2 + 1) * ny] = X;            // the row below segment t
            if (t >= 1) X = add(wga[t], mul(wde[t], X));
        }
    }
}

// the segmented march: eliminate every segment, solve the reduced systems,
// correct and substitute (never with periodic z)
template <typename T, int NYMAX, int NW, bool FULL>
static hipError_t launch_seg(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s) {
    const dim3 block(64 * NW), grid(a.slots, batch, a.zsegs);
    hipLaunchKernelGGL((k_zpipe<T, NYMAX, NW, FULL, false, 3>), grid, block, 0, s, S, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t nth = (size_t)batch * a.slots * a.ny;
    hipLaunchKernelGGL(k_zseg_reduce<T>, dim3((unsigned)((nth + 63) / 64)), dim3(64), 0, s, a, batch);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_zpipe<T, NYMAX, NW, FULL, false, 4>), grid, block, 0, s, S, a);
    return hipGetLastError();
}

template <typename T, int NYMAX, int NW, bool FULL>
static hipError_t launch_pipe(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s) {
    const dim3 block(64 * NW);
    if (a.zsegs > 0) return launch_seg<T, NYMAX, NW, FULL>(S, a, batch, s);
    if (a.zsplit > 0) {   // never with periodic z
        const dim3 grid(a.slots, batch, 2);
        hipLaunchKernelGGL((k_zpipe<T, NYMAX, NW, FULL, false, 1>), grid, block, 0, s, S, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_zpipe<T, NYMAX, NW, FULL, false, 2>), grid, block, 0, s, S, a);
        return hipGetLastError();
    }
    const dim3 grid(a.slots, batch);
    if (a.zper) hipLaunchKernelGGL((k_zpipe<T, NYMAX, NW, FULL, true, 0>), grid, block, 0, s, S, a);
    else hipLaunchKernelGGL((k_zpipe<T, NYMAX, NW, FULL, false, 0>), grid, block, 0, s, S, a);
    return hipGetLastError();
}

template <typename T, int NYMAX, int NW>
static hipError_t launch_pipe_any(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s) {
    if (pipe_full(a, NYMAX, NW)) return launch_pipe<T, NYMAX, NW, true>(S, a, batch, s);
    return launch_pipe<T, NYMAX, NW, false>(S, a, batch, s);
}

template <typename T, int RMAX, int OWN>
static hipError_t launch_mid_shape(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s) {
    const size_t lds = zmarch_lds_bytes(a.zb, a.ldy, a.ny, sizeof(cplx<T>));
    const hipError_t le = allow_dynamic_lds(reinterpret_cast<const void*>(k_zmarch<T, kZThreads, RMAX, OWN>), kZLdsBytes);
    if (le != hipSuccess) return le;
    hipLaunchKernelGGL((k_zmarch<T, kZThreads, RMAX, OWN>), dim3(a.slots, batch), dim3(kZThreads), lds, s, S, a);
    return hipGetLastError();
}

// ny <= 1024: the pipelined march (8 wavefronts; 6 for float lines of 384, 4
// for double lines over 512); longer lines: k_zmarch with 32 values per lane and
// four z entries per thread (ny <= 2048).
template <typename T>
hipError_t launch_mid(cplx<T>* S, const MidArgs<T>& a, int batch, hipStream_t s) {
    if (a.zsolver == 1 || a.zsolver == 2) return launch_mid_pcr<T>(S, a, batch, s, a.zsolver == 2);
    // segmented lines up to 256: four wavefronts, one entry per thread, 27 KB
    // of LDS in double, so that several segments' workgroups share a CU
    if (a.zsegs > 0 && a.ny <= 256) {
        if (pipe_full(a, 256, 4)) return launch_seg<T, 256, 4, true>(S, a, batch, s);
        return launch_seg<T, 256, 4, false>(S, a, batch, s);
    }
    // float lines of 384: one entry per thread, no idle lanes (measured 1.42 ->
    // 1.12 ms at 384^3 x 4; in double the 8-wavefront form is as fast)
    if constexpr (sizeof(T) == 4) {
        if (a.ny == 384) return launch_pipe_any<T, 384, 6>(S, a, batch, s);
    }
    if (a.ny <= 512) return launch_pipe_any<T, 512, 8>(S, a, batch, s);
    if (a.ny <= 1024) {
        if constexpr (sizeof(T) == 4) return launch_pipe_any<T, 1024, 8>(S, a, batch, s);
        else return launch_pipe_any<T, 1024, 4>(S, a, batch, s);
    }
    return launch_mid_shape<T, 32, 4>(S, a, batch, s);
}

template <int NYMAX, int NW, bool FULL>
static hipError_t launch_mixed(const cplx<double>* Slo, cplx<float>* S, const MidArgs<double>& ad,
                               const MidArgs<float>& af, int lo0, int nlo, int batch, hipStream_t s) {
    const dim3 block(64 * NW);
    if (af.zsplit > 0) {   // never with periodic z
        const dim3 grid(af.slots, batch, 2);
        hipLaunchKernelGGL((k_zpipe_mixed<NYMAX, NW, FULL, false, 1>), grid, block, 0, s, Slo, S, ad, af, lo0, nlo);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_zpipe_mixed<NYMAX, NW, FULL, false, 2>), grid, block, 0, s, Slo, S, ad, af, lo0, nlo);
        return hipGetLastError();
    }
    const dim3 grid(af.slots, batch);
    if (af.zper)
        hipLaunchKernelGGL((k_zpipe_mixed<NYMAX, NW, FULL, true, 0>), grid, block, 0, s, Slo, S, ad, af, lo0, nlo);
    else
        hipLaunchKernelGGL((k_zpipe_mixed<NYMAX, NW, FULL, false, 0>), grid, block, 0, s, Slo, S, ad, af, lo0, nlo);
    return hipGetLastError();
}

bool mixed_march_supported(int ny, int zsolver) { return zsolver == 0 && ny <= 1024; }

hipError_t launch_mid_mixed(const cplx<double>* Slo, cplx<float>* S, const MidArgs<double>& ad,
                            const MidArgs<float>& af, int lo0, int nlo, int batch, hipStream_t s) {
    if (nlo > 0) {
        const int nplanes = nlo * af.nz * batch;
        const size_t lds = (2 * (size_t)af.ny + (size_t)kYpreWaves * af.ldy) * sizeof(cplx<double>);
        cplx<double>* lo = const_cast<cplx<double>*>(Slo);
        const int grid = (nplanes + kYpreWaves - 1) / kYpreWaves;
        if (af.ny <= 384) {
            hipLaunchKernelGGL(k_ypre<6>, dim3(grid), dim3(64 * kYpreWaves), lds, s, lo, ad, lo0, nlo, nplanes);
        } else if (af.ny <= 512) {
            hipLaunchKernelGGL(k_ypre<8>, dim3(grid), dim3(64 * kYpreWaves), lds, s, lo, ad, lo0, nlo, nplanes);
        } else {
            const hipError_t le = allow_dynamic_lds(reinterpret_cast<const void*>(k_ypre<16>), (int)lds);
            if (le != hipSuccess) return le;
            hipLaunchKernelGGL(k_ypre<16>, dim3(grid), dim3(64 * kYpreWaves), lds, s, lo, ad, lo0, nlo, nplanes);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (af.ny == 384) {
        if (pipe_full(af, 384, 6)) return launch_mixed<384, 6, true>(Slo, S, ad, af, lo0, nlo, batch, s);
        return launch_mixed<384, 6, false>(Slo, S, ad, af, lo0, nlo, batch, s);
    }
    if (af.ny > 512) {
        if (pipe_full(af, 1024, 8)) return launch_mixed<1024, 8, true>(Slo, S, ad, af, lo0, nlo, batch, s);
        return launch_mixed<1024, 8, false>(Slo, S, ad, af, lo0, nlo, batch, s);
    }
    if (pipe_full(af, 512, 8)) return launch_mixed<512, 8, true>(Slo, S, ad, af, lo0, nlo, batch, s);
    return launch_mixed<512, 8, false>(Slo, S, ad, af, lo0, nlo, batch, s);
}

int zpipe_planes(int ny, bool dbl) {
    if (ny > 1024) return 0;
    if (!dbl && ny == 384) return 6;
    return (dbl && ny > 512) ? 4 : 8;
}

template hipError_t launch_mid<double>(cplx<double>*, const MidArgs<double>&, int, hipStream_t);
template hipError_t launch_mid<float>(cplx<float>*, const MidArgs<float>&, int, hipStream_t);

}  // namespace pp
