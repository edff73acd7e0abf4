// Device building blocks: complex arithmetic, radix-2/3/4/8 butterflies and a
// batched mixed-radix Stockham FFT over lines held in LDS.
//
// The complex DFT is the primitive every real transform of the method is built
// on (section "Boundary Conditions": pre-process, complex FFT, post-process).
// Lines of length N = 2^a 3^b sit in LDS, one line every `ldl` elements, with
// one spare slot after every 8 elements (pad()) to spread the power-of-two
// strides of the first stages over the LDS banks.
//
// Stockham step (self-sorting, decimation in time), for a stage of radix R
// after sub-transforms of length Ls have been formed, butterfly j in [0, N/R):
//     k = j mod Ls,   inputs  x[j + t N/R] * w^(t k N/(Ls R)),  t = 0..R-1
//     outputs y[(j - k) R + k + t Ls] = DFT_R(inputs)[t]
// with w = exp(-2 pi i / N) (conjugated for the inverse).  After the last
// stage the line holds the transform in natural order.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

namespace pp {

template <typename T> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };
template <typename T> using cplx = typename vec2<T>::type;

template <typename T> __host__ __device__ __forceinline__ cplx<T> mk(T re, T im) {
    cplx<T> r;
    r.x = re;
    r.y = im;
    return r;
}
// Complex helpers, generic over the two-component vector types (double2, float2).
template <typename V> __device__ __forceinline__ V cadd(V a, V b) {
    V r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename V> __device__ __forceinline__ V csub(V a, V b) {
    V r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
    V r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) {
    V r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}

// Complex value in another precision.
template <typename To, typename V> __device__ __forceinline__ cplx<To> cvt(const V& v) {
    if constexpr (std::is_same_v<V, cplx<To>>) return v;
    else return mk<To>((To)v.x, (To)v.y);
}

// Multiply by -i (forward transforms) or +i (inverse transforms).
template <bool INV, typename V> __device__ __forceinline__ V rot(V a) {
    V r;
    if (INV) {
        r.x = -a.y;
        r.y = a.x;
    } else {
        r.x = a.y;
        r.y = -a.x;
    }
    return r;
}

// floor(i / n) for 0 <= i, 1 <= n with i + n < 2^22, from inv = 1.0f / n:
// (i + 1/2) / n lies at least 1/(2n) away from an integer, and the float
// rounding error of (i + 1/2) * inv is below (i/n + 1) 2^-23 < 1/(2n).
__device__ __forceinline__ int fdiv(int i, float inv) { return (int)(((float)i + 0.5f) * inv); }

__host__ __device__ __forceinline__ int pad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int padded_len(int n) { return n + ((n - 1) >> 3); }

// Position of x[n] after the reordering that turns a DCT-II into one complex
// DFT (even-indexed samples ascending, then odd-indexed samples descending;
// Neumann subsection).  The inverse DCT-III reads its result back through the
// same map.
__device__ __forceinline__ int makhoul_pos(int n, int N) { return (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1); }

// ---------------------------------------------------------------- butterflies
template <bool INV, typename T> __device__ __forceinline__ void bfly2(cplx<T>* v) {
    cplx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <bool INV, typename T> __device__ __forceinline__ void bfly4(cplx<T>* v) {
    cplx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cplx<T> s13 = cadd(v[1], v[3]), d13 = rot<INV>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

template <bool INV, typename T> __device__ __forceinline__ void bfly8(cplx<T>* v) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    bfly4<INV, T>(e);
    bfly4<INV, T>(o);
    const T r = T(0.70710678118654752440);  // 1/sqrt(2)
    // o1 * w^1, o2 * w^2, o3 * w^3 with w = exp(-+ i pi / 4)
    cplx<T> o1 = INV ? mk<T>((o[1].x - o[1].y) * r, (o[1].x + o[1].y) * r)
                     : mk<T>((o[1].x + o[1].y) * r, (o[1].y - o[1].x) * r);
    cplx<T> o2 = rot<INV>(o[2]);
    cplx<T> o3 = INV ? mk<T>((-o[3].x - o[3].y) * r, (o[3].x - o[3].y) * r)
                     : mk<T>((o[3].y - o[3].x) * r, (-o[3].x - o[3].y) * r);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <bool INV, typename T> __device__ __forceinline__ void bfly3(cplx<T>* v) {
    const T h = T(0.86602540378443864676);  // sqrt(3)/2
    cplx<T> t1 = cadd(v[1], v[2]);
    cplx<T> t2 = mk<T>(v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y);
    cplx<T> dd = csub(v[1], v[2]);
    cplx<T> t3 = rot<INV>(mk<T>(h * dd.x, h * dd.y));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
}

template <int R, bool INV, typename T> __device__ __forceinline__ void bfly(cplx<T>* v) {
    if constexpr (R == 2) bfly2<INV, T>(v);
    else if constexpr (R == 3) bfly3<INV, T>(v);
    else if constexpr (R == 4) bfly4<INV, T>(v);
    else bfly8<INV, T>(v);
}

// Radix plan of one transform length, fixed on the host.
struct FftDesc {
    int n;
    int nstages;
    int radix[16];
};

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Streaming accesses (non-temporal: the caches do not keep the line) for data
// a kernel touches once and that no later kernel reads soon enough to find in
// a cache.  Used where measured to help: the source rows of the forward x
// kernel, the solution rows of the inverse, the refinement residual's source
// and output, and the float spectra written by the forward x kernel.
// (Complex values go through the two-element native vector of their type.)
template <typename V> __device__ __forceinline__ V ld_stream(const V* p) {
    if constexpr (std::is_arithmetic_v<V>) {
        return __builtin_nontemporal_load(p);
    } else {
        using N = typename V::Native_vec_;
        const N n = __builtin_nontemporal_load(reinterpret_cast<const N*>(p));
        V r;
        r.x = n[0];
        r.y = n[1];
        return r;
    }
}
template <typename V> __device__ __forceinline__ void st_stream(V* p, const V& v) {
    if constexpr (std::is_arithmetic_v<V>) {
        __builtin_nontemporal_store(v, p);
    } else {
        using N = typename V::Native_vec_;
        const N n = {v.x, v.y};
        __builtin_nontemporal_store(n, reinterpret_cast<N*>(p));
    }
}

// Order this wavefront's LDS accesses: LDS instructions of one wavefront are
// performed in issue order, so a compiler-level fence at wavefront scope is
// all a wave needs between writing and re-reading its own LDS region.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup barrier that orders LDS accesses only: the wavefront's LDS
// operations complete, then all wavefronts meet.  Unlike __syncthreads() it
// does not wait for outstanding global loads, which the pipelined kernels keep
// in flight across barriers.  The memory clobber keeps the compiler from moving
// memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Wavefront-private Stockham stage: the 64 lanes of one wave transform one
// line in place (all of the wave's reads precede its writes in program order).
// MAXB = butterflies per lane = ceil(N / R / 64).
//
// Twiddles are packed by stage: the stage whose sub-transforms have length Ls
// (radix R) reads w_N^(t k N / (Ls R)), t = 1..R-1, k = 0..Ls-1, at index
// t * Ls + k - 1, so the stages occupy [Ls - 1, R Ls - 1) one after another
// (N - 1 entries in all) and the lanes of a stage, which run over consecutive
// k, read consecutive entries (no LDS bank conflicts).
template <int R, int MAXB, bool INV, typename T>
__device__ __forceinline__ void wfft_stage(cplx<T>* line, int N, int Ls, const cplx<T>* tw, int lane) {
    const int nbf = N / R;
    const float inv_ls = 1.0f / (float)Ls;
    cplx<T> v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int j = lane + 64 * i;
        dst[i] = -1;
        if (j < nbf) {
            const int k = j - fdiv(j, inv_ls) * Ls;
#pragma unroll
            for (int t = 0; t < R; ++t) v[i][t] = line[pad(j + t * nbf)];
            if (Ls > 1) {
#pragma unroll
                for (int t = 1; t < R; ++t) {
                    const cplx<T> w = tw[t * Ls + k - 1];
                    v[i][t] = INV ? cmulc(v[i][t], w) : cmul(v[i][t], w);
                }
            }
            bfly<R, INV, T>(v[i]);
            dst[i] = (j - k) * R + k;
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        if (dst[i] >= 0) {
#pragma unroll
            for (int t = 0; t < R; ++t) line[pad(dst[i] + t * Ls)] = v[i][t];
        }
    }
    wave_lds_sync();
}

// One line of d.n <= 64 * EPL complex values, transformed by one wavefront.
template <int EPL, bool INV, typename T>
__device__ __forceinline__ void wfft(cplx<T>* line, const FftDesc& d, const cplx<T>* tw, int lane) {
    int Ls = 1;
    for (int s = 0; s < d.nstages; ++s) {
        const int R = d.radix[s];
        if (R == 8) wfft_stage<8, cdiv(EPL, 8), INV, T>(line, d.n, Ls, tw, lane);
        else if (R == 4) wfft_stage<4, cdiv(EPL, 4), INV, T>(line, d.n, Ls, tw, lane);
        else if (R == 3) wfft_stage<3, cdiv(EPL, 3), INV, T>(line, d.n, Ls, tw, lane);
        else wfft_stage<2, cdiv(EPL, 2), INV, T>(line, d.n, Ls, tw, lane);
        Ls *= R;
    }
}

// 512-point transform of one line by one wavefront: the radix plan of 512 is
// three radix-8 Stockham stages (sub-transform lengths Ls = 1, 8, 64).  In
// every stage lane j reads elements j + 64 t; the first stage has no
// twiddles, and the last writes its outputs back to j + 64 t, the natural
// order.  So a line whose elements y = lane + 64 t sit in a lane's registers
// can enter the first stage without an LDS round trip, and the last stage can
// hand its outputs to the caller in registers in the same order.  A lane's
// twiddles of stages 2 and 3 are the same for every line: a kernel with
// registers to spare keeps them there (Tw512Reg), others read them from the
// LDS table (Tw512Lds).
template <typename T> struct Tw512Reg {
    cplx<T> r2[7], r3[7];
    __device__ __forceinline__ cplx<T> s2(int t) const { return r2[t - 1]; }
    __device__ __forceinline__ cplx<T> s3(int t) const { return r3[t - 1]; }
};

// packed table (see wfft_stage): stage Ls, factor t, index k at t Ls + k - 1
template <typename T> struct Tw512Lds {
    const cplx<T>* tw;
    int lane;
    __device__ __forceinline__ cplx<T> s2(int t) const { return tw[t * 8 + (lane & 7) - 1]; }
    __device__ __forceinline__ cplx<T> s3(int t) const { return tw[t * 64 + lane - 1]; }
};

template <typename T> __device__ __forceinline__ Tw512Reg<T> tw512_regs(const cplx<T>* tw, int lane) {
    const Tw512Lds<T> src{tw, lane};
    Tw512Reg<T> w;
#pragma unroll
    for (int t = 1; t < 8; ++t) {
        w.r2[t - 1] = src.s2(t);
        w.r3[t - 1] = src.s3(t);
    }
    return w;
}

// stage 1 on values in registers (v[t] = element lane + 64 t), result to the line
template <bool INV, typename T> __device__ __forceinline__ void w512_first(cplx<T> (&v)[8], cplx<T>* line, int lane) {
    bfly8<INV, T>(v);
#pragma unroll
    for (int t = 0; t < 8; ++t) line[pad(lane * 8 + t)] = v[t];
    wave_lds_sync();
}

// stage 1 on the line, in place
template <bool INV, typename T> __device__ __forceinline__ void w512_first_lds(cplx<T>* line, int lane) {
    cplx<T> v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = line[pad(lane + 64 * t)];
    wave_lds_sync();
    w512_first<INV, T>(v, line, lane);
}

// stage 2 on the line, in place
template <bool INV, typename T, typename TW>
__device__ __forceinline__ void w512_second(cplx<T>* line, const TW& w, int lane) {
    cplx<T> v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = line[pad(lane + 64 * t)];
#pragma unroll
    for (int t = 1; t < 8; ++t) v[t] = INV ? cmulc(v[t], w.s2(t)) : cmul(v[t], w.s2(t));
    bfly8<INV, T>(v);
    const int k = lane & 7;
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < 8; ++t) line[pad((lane - k) * 8 + k + 8 * t)] = v[t];
    wave_lds_sync();
}

// stage 3 from the line; the outputs stay in registers (v[t] = element lane + 64 t)
template <bool INV, typename T, typename TW>
__device__ __forceinline__ void w512_last(const cplx<T>* line, const TW& w, int lane, cplx<T> (&v)[8]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = line[pad(lane + 64 * t)];
#pragma unroll
    for (int t = 1; t < 8; ++t) v[t] = INV ? cmulc(v[t], w.s3(t)) : cmul(v[t], w.s3(t));
    bfly8<INV, T>(v);
}

// Maximum that keeps a NaN from either argument (fmax drops it), so that a
// non-finite source or solution reaches the scalars the host checks.
__device__ __forceinline__ double nmax(double a, double b) { return (b > a || b != b) ? b : a; }

// Sum of a double over the block (wave64 shuffles, then LDS across waves).
// Result valid in thread 0.
template <int NTH> __device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < NTH / 64; ++w) s += red[w];
    }
    __syncthreads();
    return s;
}

template <int NTH> __device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nmax(v, __shfl_down(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < NTH / 64; ++w) s = nmax(s, red[w]);
    }
    __syncthreads();
    return s;
}

}  // namespace pp
