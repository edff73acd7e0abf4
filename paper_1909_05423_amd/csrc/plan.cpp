// Plan creation, table construction, workspace layout and the launch sequences
// behind the C ABI of include/ppsolve.h.
//
// Host-side numerics (all double, angles reduced exactly over the integers and
// evaluated in long double before rounding):
//   * FFT twiddles (powers of exp(-2 pi i / N), packed by stage) and the DCT twiddles exp(-i pi k / (2N));
//   * the 1-D eigenvalues of Table eig, written -4 sin^2(t/2) / h^2 (equal to
//     the table's -2 + 2 cos(t), without its cancellation at small t);
//   * the reciprocal pivots of every z-system (section "Solution of the
//     Resulting Tridiagonal Matrices", Algorithm Thomas for Toeplitz Matrices)
//     up to the index where they stop changing in the solve's precision.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/ppsolve.h"
#include "pp_kernels.hpp"

using pp::cplx;

// Host tables of one precision and their byte offsets inside the blob.
struct Tables {
    std::vector<unsigned char> blob;
    size_t t_twx = 0, t_mkx = 0, t_twy = 0, t_mky = 0, t_rowoff = 0, t_lmax = 0, t_winf = 0, t_wlast = 0, t_wrows = 0;
    size_t t_elen = 0;
    size_t t_bmid = 0;   // interior z diagonal per (slot, entry, part)
    // split march: the lower half's pivots (by distance from the bottom row) and the meeting rows
    size_t t_browoff = 0, t_belen = 0, t_bwinf = 0, t_bwrows = 0, t_meet = 0;
    // segmented march: fresh pivots of a segment starting inside the column,
    // its forward-eliminated first unit vector (rho), the last segment's
    // last-row values, and the end values of the segments' responses
    size_t t_frowoff = 0, t_felen = 0, t_fwinf = 0, t_fwrows = 0, t_flast = 0;
    size_t t_rrowoff = 0, t_relen = 0, t_rrows = 0, t_rholast = 0, t_segk = 0;
    // periodic z (Sherman-Morrison)
    size_t t_aelen = 0, t_qelen = 0;
    size_t t_aoff = 0, t_alen = 0, t_arows = 0, t_qoff = 0, t_qlen = 0, t_qrows = 0, t_qlast = 0, t_invden = 0,
           t_invgam = 0;
    size_t table_rows = 0;
};

struct pp_plan_s {
    int nx = 0, ny = 0, nz = 0, batch = 0;
    char bc[6] = {0};
    double h[3] = {0, 0, 0};
    pp_dtype dtype = PP_F64;
    pp_gauge gauge = PP_GAUGE_MEAN;
    double ir_tol = 1e-13;
    int ir_max = 8;
    // derived
    int bx = 0, by = 0, bz0 = 0, bz1 = 0;
    bool singular = false;
    int slots = 0;
    size_t elem = 0;  // bytes of one complex value of the solve precision
    pp::FftDesc fx{}, fy{};
    int ty = 0, ldl = 0, ldy = 0, zb = 0;
    size_t nper = 0;  // upper bound of the x-kernel partial records per batch entry
    // tables (uploaded into the workspace): tb[0] in the solve precision; for
    // PP_F32_REFINED also tb[1] in double (the double-arithmetic x transform and
    // the slots the mixed march runs in double)
    Tables tb[2];
    int ntab = 1;
    int zsolver = 0;     // 0 Thomas (fused march), 1 PCR, 2 CR-P
    // split march (non-periodic z, pipelined forms): first row of the lower
    // half, a multiple of the march's chunk; 0 if the shape has no split form.
    // Used when the columns alone would leave compute units idle.
    int zsplit = 0;
    int zsplit_mode = 0;   // pp_zsplit
    // segmented march (few columns, long z): zsegs segments of zseglen rows
    // (the last one the remainder); 0 if the plan has no segmented form
    int zsegs = 0, zseglen = 0;
    // largest 1 / |1 - v w| of the split march's meeting rows (the factor by
    // which they amplify rounding): near-singular z-systems (the zero mode,
    // the lowest wavenumbers of long columns with Neumann or periodic x, y)
    // make it large, and the automatic choice then keeps one march per column
    double split_gmax = 0.0;
    // refined solve: slots lo0 .. lo0+nlo-1 kept in double by the x transform and the z march
    int lo0 = 0, nlo = 0;
    // the first correction's size may stand for the refinement's contraction
    // (see set_mixed_slots and run_refined)
    bool fast_stop = false;
    // workspace layout (byte offsets): o_tab[i] holds tb[i]; o_S the spectral
    // array; refined: o_r the float residual, o_u0 the float first solution,
    // o_lo the double slots
    size_t o_scalars = 0, o_partial = 0, o_tab[2] = {0, 0}, o_S = 0, o_r = 0, o_u0 = 0, o_lo = 0, ws_bytes = 0;
    size_t o_zb[2] = {0, 0};   // split march: the halves' last eliminated values, per table set
    size_t o_seg = 0;          // segmented march: segment end values, reduction scratch, couplings
    unsigned long long serial = 0;   // identifies the plan in the workspace registry
    // last call
    void* last_ws = nullptr;
    hipStream_t last_stream = nullptr;
    int last_iters = 0;
    double last_rel = 0.0;
    bool last_projected = false;
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;               // created lazily, reused
    std::vector<std::pair<int, int>> marks;        // (event index, kernel group of the next launch)
    double kms[4] = {0, 0, 0, 0};
    int kcount[4] = {0, 0, 0, 0};
    ~pp_plan_s() {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
};

namespace {

constexpr size_t kAlign = 256;
// segmented march: at most this many segments per column, and segments enough
// for this many workgroups (the compute units of an MI355X)
constexpr int kMaxSegments = pp::kMaxZSegments;
constexpr long long kSegTargetColumns = 256;
// y lines up to 256 run a march of four wavefronts (27 KB of LDS in double),
// several workgroups per CU: segments enough for three per CU in double (the
// registers it takes) and four in float
constexpr long long kSegTargetNarrowF64 = 768, kSegTargetNarrowF32 = 1024;
// the automatic choice splits columns only where the meeting rows amplify
// rounding by at most this much (measured: errors near 2.5e-15 times it)
constexpr double kSplitGMax = 256.0;

// Which plan's tables each workspace holds: workspace base pointer -> serial
// number of the plan that last uploaded its tables there.  A solve re-uploads
// the tables when the workspace it is given was last used by another plan
// (two plans sharing one workspace, the fixed buffer of pp_solve_noalloc).
std::mutex g_ws_mu;
std::map<const void*, unsigned long long> g_ws_owner;
unsigned long long g_next_serial = 1;

bool tables_present(const pp_plan p, const void* ws) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    const auto it = g_ws_owner.find(ws);
    return it != g_ws_owner.end() && it->second == p->serial;
}
void tables_uploaded(const pp_plan p, const void* ws) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    g_ws_owner[ws] = p->serial;
}
void forget_plan(const pp_plan p) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    for (auto it = g_ws_owner.begin(); it != g_ws_owner.end();) {
        if (it->second == p->serial) it = g_ws_owner.erase(it);
        else ++it;
    }
}
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int bc_code(char c) {
    switch (c) {
        case 'P': return pp::BC_P;
        case 'N': return pp::BC_N;
        case 'D': return pp::BC_D;
        default: return -1;
    }
}

bool factor23(int n) {
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// Radix plan: as many radix-8 stages as possible (two radix-4 stages instead
// of an 8 and a 2), then radix 3.
pp::FftDesc radix_plan(int n) {
    pp::FftDesc d{};
    d.n = n;
    int a = 0, b = 0, m = n;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    int s = 0;
    int n8 = a / 3, rem = a % 3;
    if (rem == 1 && n8 >= 1) {
        for (int i = 0; i < n8 - 1; ++i) d.radix[s++] = 8;
        d.radix[s++] = 4;
        d.radix[s++] = 4;
    } else {
        for (int i = 0; i < n8; ++i) d.radix[s++] = 8;
        if (rem == 1) d.radix[s++] = 2;
        if (rem == 2) d.radix[s++] = 4;
    }
    for (int i = 0; i < b; ++i) d.radix[s++] = 3;
    d.nstages = s;
    return d;
}

const long double kPi = 3.141592653589793238462643383279502884L;

// cos and sin of pi * num / den with num reduced modulo 2 den first.
void cos_sin_pi(long long num, long long den, double* c, double* s) {
    long long r = num % (2 * den);
    if (r < 0) r += 2 * den;
    const long double t = kPi * (long double)r / (long double)den;
    *c = (double)cosl(t);
    *s = (double)sinl(t);
}

// Table eig for one direction: mode k of n cells, spacing h.
double eigenvalue(int kind, int k, int n, double h) {
    long long num = 0;
    if (kind == pp::BC_P) num = 2LL * k;
    else if (kind == pp::BC_N) num = k;
    else num = (long long)k + 1;
    // -2 + 2 cos(pi num / n) = -4 sin^2(pi num / (2 n))
    long long r = num % (2LL * n);
    const long double half = kPi * (long double)r / (2.0L * (long double)n);
    const long double s = sinl(half);
    return (double)(-4.0L * s * s / ((long double)h * (long double)h));
}

template <typename T> struct Emit {
    std::vector<unsigned char>& blob;
    size_t put(size_t bytes) {
        const size_t off = align_up(blob.size());
        blob.resize(off + bytes, 0);
        return off;
    }
    cplx<T>* cp(size_t off) { return reinterpret_cast<cplx<T>*>(blob.data() + off); }
};

// Reciprocal pivots of one z line.  body = w_0 .. w_{nz-2} until the value
// stops changing; wl = w_{nz-1}; tail = first index from which the rounded
// body value equals the rounded value at nz-2.
//
// Periodic z (Thomas subsection: the cyclic system by Sherman-Morrison).  With
// gamma = -b the cyclic matrix is T' + v v'^T, v = (gamma, 0, .., 0, 1),
// v' = (1, 0, .., 0, 1/gamma), where T' is tridiagonal with first diagonal
// b - gamma = 2b and last diagonal b - 1/gamma.  Its solution is
// u = y - c q with y = T'^{-1} d, q = T'^{-1} v and
// c = (y_0 + y_{n-1}/gamma) / (1 + q_0 + q_{n-1}/gamma).  The kernels eliminate
// with the pivots of T'; y_{n-1} is the last eliminated value, and
// y_0 = sum_z alpha_z d_z with alpha = T'^{-1} e_0 (T' is symmetric), so c is
// known when the march turns; on the way down q_z = qp_z - w_z q_{z+1} from
// the forward-eliminated qp = (v after elimination).  alpha and qp decay
// geometrically away from z = 0 and are stored up to where they fall below
// 2^-60 of their largest value.  The pinned zero-mode line of a singular
// problem (u_0 = 0, section "Well-posedness") is an ordinary tridiagonal
// system and keeps alpha = qp = 0, 1/den = 0, so c = 0.
template <typename T> struct Line {
    std::vector<T> body;
    T winf = 0, wlast = 0;
    int tail = 0;
    std::vector<T> alpha, qp;       // periodic z only
    T qlast = 0, inv_den = 0, inv_gamma = 0;
};

template <typename T> static int significant_prefix(const std::vector<double>& v) {
    double mx = 0.0;
    for (double x : v) mx = std::max(mx, std::fabs(x));
    int L = (int)v.size();
    while (L > 0 && std::fabs(v[L - 1]) <= mx * 0x1p-60) --L;
    return L;
}

template <typename T> void periodic_extras(double bmid, int nz, const std::vector<double>& w, Line<T>* out) {
    const double gamma = -bmid;
    std::vector<double> qp(nz), q(nz), ap(nz), al(nz);
    qp[0] = gamma * w[0];
    ap[0] = w[0];
    for (int z = 1; z < nz; ++z) {
        const double vz = (z == nz - 1) ? 1.0 : 0.0;
        qp[z] = (vz - qp[z - 1]) * w[z];
        ap[z] = (0.0 - ap[z - 1]) * w[z];
    }
    q[nz - 1] = qp[nz - 1];
    al[nz - 1] = ap[nz - 1];
    for (int z = nz - 2; z >= 0; --z) {
        q[z] = qp[z] - w[z] * q[z + 1];
        al[z] = ap[z] - w[z] * al[z + 1];
    }
    out->qlast = (T)qp[nz - 1];
    out->inv_gamma = (T)(1.0 / gamma);
    out->inv_den = (T)(1.0 / (1.0 + q[0] + q[nz - 1] / gamma));
    std::vector<double> qbody(qp.begin(), qp.end() - 1);   // the last value is qlast
    const int Lq = significant_prefix<T>(qbody);
    const int La = significant_prefix<T>(al);
    out->qp.assign(qbody.begin(), qbody.begin() + Lq);
    out->alpha.assign(al.begin(), al.begin() + La);
}

// krow >= 0: *wk = the reciprocal pivot of row krow in double (krow <= nz - 2;
// the upper half's last row in a split march).
template <typename T>
void pivots(double lam, int nz, double hz, int bz0, int bz1, bool pinned, Line<T>* out, int krow = -1,
            double* wk = nullptr) {
    const double bmid = -2.0 + hz * hz * lam;
    out->alpha.clear();
    out->qp.clear();
    out->qlast = out->inv_den = out->inv_gamma = 0;
    if (bz0 == pp::BC_P && !pinned) {
        // T' of the Sherman-Morrison splitting (nz >= 3): first diagonal 2b, last b + 1/b
        std::vector<double> w(nz);
        w[0] = 1.0 / (2.0 * bmid);
        for (int z = 1; z < nz - 1; ++z) w[z] = 1.0 / (bmid - w[z - 1]);
        w[nz - 1] = 1.0 / ((bmid + 1.0 / bmid) - w[nz - 2]);
        periodic_extras<T>(bmid, nz, w, out);
        out->wlast = (T)w[nz - 1];
        out->winf = (T)w[nz - 2];
        int L = nz - 1;
        while (L > 0 && (T)w[L - 1] == out->winf) --L;
        out->tail = L;
        out->body.resize(L);
        for (int i = 0; i < L; ++i) out->body[i] = (T)w[i];
        return;
    }
    // the pinned zero mode of a periodic z direction: rows 1..n-1 with u_0 = 0,
    // interior diagonal also in the last row (its wrap-around neighbour is u_0)
    const double d0 = (bz0 == pp::BC_D) ? -1.0 : 1.0;
    const double d1 = (bz1 == pp::BC_P) ? 0.0 : (bz1 == pp::BC_D) ? -1.0 : 1.0;
    out->body.clear();
    if (nz == 1) {
        out->wlast = pinned ? T(0) : (T)(1.0 / (bmid + d0 + d1));
        out->winf = 0;
        out->tail = 0;
        return;
    }
    std::vector<double> seq;
    seq.reserve(64);
    double prev = pinned ? 0.0 : 1.0 / (bmid + d0);
    seq.push_back(prev);
    for (int z = 1; z <= nz - 2; ++z) {
        const double w = 1.0 / (bmid - prev);
        seq.push_back(w);
        if (w == prev) break;  // fixed point: every later body value is the same
        prev = w;
    }
    const double wend = seq.back();  // value at index nz-2
    if (krow >= 0 && wk) *wk = seq[std::min((size_t)krow, seq.size() - 1)];
    out->wlast = (T)(1.0 / ((bmid + d1) - wend));
    out->winf = (T)wend;
    int L = (int)seq.size();
    while (L > 0 && (T)seq[L - 1] == out->winf) --L;
    out->tail = L;
    out->body.resize(L);
    for (int i = 0; i < L; ++i) out->body[i] = (T)seq[i];
}

// The lower half of a split march eliminates upward from the bottom face: the
// same recurrence with the end rows exchanged, v_j the reciprocal pivot of row
// nz-1-j for j = 0 .. jmax (stored up to convergence like the top-down
// pivots); *vk = v_jmax in double (row zsplit).
template <typename T> void bottom_pivots(double lam, int nz, double hz, int bz1, int jmax, Line<T>* out, double* vk) {
    const double bmid = -2.0 + hz * hz * lam;
    const double d1 = (bz1 == pp::BC_D) ? -1.0 : 1.0;
    out->alpha.clear();
    out->qp.clear();
    std::vector<double> seq;
    seq.reserve(64);
    double prev = 1.0 / (bmid + d1);
    seq.push_back(prev);
    for (int j = 1; j <= jmax; ++j) {
        const double v = 1.0 / (bmid - prev);
        seq.push_back(v);
        if (v == prev) break;   // fixed point
        prev = v;
    }
    *vk = seq.back();
    out->winf = (T)seq.back();
    out->wlast = out->winf;
    int L = (int)seq.size();
    while (L > 0 && (T)seq[L - 1] == out->winf) --L;
    out->tail = L;
    out->body.resize(L);
    for (int i = 0; i < L; ++i) out->body[i] = (T)seq[i];
}

// Segmented march (section "Solution of the Resulting Tridiagonal Matrices",
// the Thomas algorithm run on pieces of each z-system): segment s of nseg
// holds rows [s L, s L + len_s) and is eliminated on its own ("fresh": the
// coupling to the rows outside is moved to the right-hand side), with the
// global top pivots in segment 0 and the pivots of a segment that starts with
// the interior diagonal elsewhere (the last segment's last row with the bottom
// face).  Per line: those fresh pivots (stored up to convergence), rho =
// the fresh elimination of the segment's first unit vector (the effect of the
// coupling above it; stored until negligible), the last segment's last-row
// pivot and rho, and for the first, interior and last segment the first and
// last values of p = T_s^{-1} e_first and q = T_s^{-1} e_last, which link the
// segments' end values in the reduced system.
template <typename T> struct SegLine {
    std::vector<T> fbody, rho;
    T finf = 0, flast = 0, rholast = 0;
    int ftail = 0;
    double k[3][4] = {{0}};   // class (first, interior, last) x (p_first, p_last, q_first, q_last)
};

static void seg_ends(const std::vector<double>& piv, double* k) {
    const int L = (int)piv.size();
    std::vector<double> rho(L), pv(L), qv(L);
    for (int j = 0; j < L; ++j) rho[j] = (j == 0) ? piv[0] : -piv[j] * rho[j - 1];
    pv[L - 1] = rho[L - 1];
    for (int j = L - 2; j >= 0; --j) pv[j] = rho[j] - piv[j] * pv[j + 1];
    qv[L - 1] = piv[L - 1];
    for (int j = L - 2; j >= 0; --j) qv[j] = -piv[j] * qv[j + 1];
    k[0] = pv[0];
    k[1] = pv[L - 1];
    k[2] = qv[0];
    k[3] = qv[L - 1];
}

template <typename T>
void seg_line(double lam, int nz, double hz, int bz0, int bz1, bool pinned, int L, int nseg, SegLine<T>* out) {
    const double bmid = -2.0 + hz * hz * lam;
    const double d0 = (bz0 == pp::BC_D) ? -1.0 : 1.0;
    const double d1 = (bz1 == pp::BC_D) ? -1.0 : 1.0;
    const int Llast = nz - (nseg - 1) * L;
    // first segment: the global top pivots
    std::vector<double> pf(L);
    pf[0] = pinned ? 0.0 : 1.0 / (bmid + d0);
    for (int j = 1; j < L; ++j) pf[j] = 1.0 / (bmid - pf[j - 1]);
    seg_ends(pf, out->k[0]);
    // interior segments: fresh pivots from the interior diagonal
    std::vector<double> fi(L);
    fi[0] = 1.0 / bmid;
    for (int j = 1; j < L; ++j) fi[j] = 1.0 / (bmid - fi[j - 1]);
    seg_ends(fi, out->k[1]);
    // last segment: the same, its last row with the bottom face
    std::vector<double> fl(fi.begin(), fi.begin() + Llast);
    fl[Llast - 1] = 1.0 / ((bmid + d1) - (Llast > 1 ? fi[Llast - 2] : 0.0));
    seg_ends(fl, out->k[2]);
    out->flast = (T)fl[Llast - 1];
    // stored fresh pivots: up to the value at L - 1 (rows past the tail read finf)
    out->finf = (T)fi[L - 1];
    int tail = L;
    while (tail > 0 && (T)fi[tail - 1] == out->finf) --tail;
    out->ftail = tail;
    out->fbody.assign(fi.begin(), fi.begin() + tail);
    // rho of the interior pivots, until negligible; the last segment's last row apart
    std::vector<double> rho(L);
    double mx = 0.0;
    for (int j = 0; j < L; ++j) {
        rho[j] = (j == 0) ? fi[0] : -fi[j] * rho[j - 1];
        mx = std::max(mx, std::fabs(rho[j]));
    }
    int rl = L;
    while (rl > 0 && std::fabs(rho[rl - 1]) <= mx * 0x1p-60) --rl;
    out->rho.resize(rl);
    for (int j = 0; j < rl; ++j) out->rho[j] = (T)rho[j];
    out->rholast = (T)((Llast > 1) ? -fl[Llast - 1] * rho[Llast - 2] : fl[0]);
}

template <typename T> void build_tables(pp_plan p, Tables& tb) {
    tb.blob.clear();
    Emit<T> em{tb.blob};
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    // FFT twiddles packed by stage (the layout the wavefront FFT reads): the
    // stage with sub-transform length Ls and radix R holds exp(-2 pi i t k step / n),
    // step = n / (Ls R), at index t Ls + k - 1 (t = 1..R-1, k = 0..Ls-1)
    auto twiddles = [&](const pp::FftDesc& fd, size_t* tw, size_t* mkt) {
        const int n = fd.n;
        *tw = em.put(sizeof(cplx<T>) * n);
        em.cp(*tw)[n - 1] = pp::mk<T>(T(1), T(0));   // unused
        long long Ls = 1;
        for (int st = 0; st < fd.nstages; ++st) {
            const int R = fd.radix[st];
            const long long step = n / (Ls * R);
            for (int t = 1; t < R; ++t)
                for (long long k = 0; k < Ls; ++k) {
                    double c, s;
                    cos_sin_pi(2LL * t * k * step, n, &c, &s);
                    em.cp(*tw)[t * Ls + k - 1] = pp::mk<T>((T)c, (T)-s);
                }
            Ls *= R;
        }
        *mkt = em.put(sizeof(cplx<T>) * n);
        for (int k = 0; k < n; ++k) {
            double c, s;
            cos_sin_pi(k, 2LL * n, &c, &s);  // exp(-i pi k / (2 n))
            em.cp(*mkt)[k] = pp::mk<T>((T)c, (T)-s);
        }
    };
    twiddles(p->fx, &tb.t_twx, &tb.t_mkx);
    twiddles(p->fy, &tb.t_twy, &tb.t_mky);

    std::vector<double> lamx(nx), lamy(ny);
    for (int k = 0; k < nx; ++k) lamx[k] = eigenvalue(p->bx, k, nx, p->h[0]);
    for (int k = 0; k < ny; ++k) lamy[k] = eigenvalue(p->by, k, ny, p->h[1]);

    // kx of part `part` of slot m (-1: padding column of an odd nx)
    auto kx_of = [&](int m, int part) -> int {
        if (p->bx == pp::BC_P) {
            if (m == 0) return part == 0 ? 0 : ((nx % 2 == 0) ? nx / 2 : -1);
            return m;
        }
        const int k = 2 * m + part;
        if (k >= nx) return -1;
        return p->bx == pp::BC_D ? nx - 1 - k : k;  // DST columns are stored reversed
    };

    const int slots = p->slots;
    std::vector<int> rowoff(slots), lmax(slots), elen((size_t)slots * ny);
    std::vector<T> winf((size_t)slots * ny * 2), wlast((size_t)slots * ny * 2);
    std::vector<std::vector<Line<T>>> lines(slots);
    // split march: the lower half's lines and, per (slot, entry, part), the
    // meeting rows' pivots w (row zsplit-1, top-down), v (row zsplit,
    // bottom-up) and 1 / (1 - v w), all from double
    const int ks = p->zsplit;
    std::vector<std::vector<Line<T>>> blines(ks > 0 ? slots : 0);
    std::vector<T> meet(ks > 0 ? (size_t)slots * ny * 6 : 0);
    const int nseg = p->zsegs;
    std::vector<std::vector<SegLine<T>>> slines(nseg > 0 ? slots : 0);
    size_t rows = 0;
    for (int m = 0; m < slots; ++m) {
        const bool pairslot = (p->bx != pp::BC_P) || (m == 0);
        const bool sep = (p->by == pp::BC_P) && pairslot;
        lines[m].resize((size_t)ny * 2);
        int lm = 0;
        for (int e = 0; e < ny; ++e) {
            for (int part = 0; part < 2; ++part) {
                int kx, ky;
                if (sep && e != 0 && 2 * e != ny) {
                    kx = kx_of(m, e < ny - e ? 0 : 1);
                    ky = e;  // periodic eigenvalues are symmetric in ky <-> ny-ky
                } else {
                    kx = kx_of(m, part);
                    ky = (p->by == pp::BC_D) ? ny - 1 - e : e;  // DST entries are stored reversed
                }
                Line<T>& ln = lines[m][(size_t)e * 2 + part];
                double wk = 0.0, vk = 0.0;
                if (kx < 0) {
                    ln.body.clear();
                    ln.winf = 0;
                    ln.wlast = 0;
                    ln.tail = 0;
                } else {
                    const bool pinned = p->singular && m == 0 && e == 0 && part == 0;
                    pivots<T>(lamx[kx] + lamy[ky], nz, p->h[2], p->bz0, p->bz1, pinned, &ln, ks - 1, &wk);
                }
                if (nseg > 0) {
                    if (slines[m].empty()) slines[m].resize((size_t)ny * 2);
                    SegLine<T>& sl = slines[m][(size_t)e * 2 + part];
                    if (kx >= 0) {
                        const bool pinned = p->singular && m == 0 && e == 0 && part == 0;
                        seg_line<T>(lamx[kx] + lamy[ky], nz, p->h[2], p->bz0, p->bz1, pinned, p->zseglen, nseg, &sl);
                    } else {
                        // padding part: zero right-hand side; any non-singular values
                        sl.k[0][3] = sl.k[1][3] = sl.k[2][3] = 0.0;
                    }
                }
                if (ks > 0) {
                    if (blines[m].empty()) blines[m].resize((size_t)ny * 2);
                    Line<T>& bl = blines[m][(size_t)e * 2 + part];
                    if (kx >= 0) bottom_pivots<T>(lamx[kx] + lamy[ky], nz, p->h[2], p->bz1, nz - 1 - ks, &bl, &vk);
                    T* mt = meet.data() + ((size_t)m * ny + e) * 6;
                    mt[part] = (T)wk;
                    mt[2 + part] = (T)vk;
                    mt[4 + part] = (T)(1.0 / (1.0 - vk * wk));
                    if (kx >= 0) p->split_gmax = std::max(p->split_gmax, std::fabs(1.0 / (1.0 - vk * wk)));
                }
                winf[((size_t)m * ny + e) * 2 + part] = ln.winf;
                wlast[((size_t)m * ny + e) * 2 + part] = ln.wlast;
                lm = std::max(lm, ln.tail);
                int& el = elen[(size_t)m * ny + e];
                el = part ? std::max(el, ln.tail) : ln.tail;
            }
        }
        rowoff[m] = (int)rows;
        lmax[m] = lm;
        rows += lm;
    }
    tb.table_rows = rows;
    tb.t_rowoff = em.put(sizeof(int) * slots);
    std::memcpy(tb.blob.data() + tb.t_rowoff, rowoff.data(), sizeof(int) * slots);
    tb.t_lmax = em.put(sizeof(int) * slots);
    std::memcpy(tb.blob.data() + tb.t_lmax, lmax.data(), sizeof(int) * slots);
    // per-entry lengths: a lane reads its table row only while its entry's
    // pivots still change, so slots with a few slowly converging entries (the
    // smallest wavenumbers) do not read whole rows for most of z
    tb.t_elen = em.put(sizeof(int) * elen.size());
    std::memcpy(tb.blob.data() + tb.t_elen, elen.data(), sizeof(int) * elen.size());
    tb.t_winf = em.put(sizeof(T) * winf.size());
    std::memcpy(tb.blob.data() + tb.t_winf, winf.data(), sizeof(T) * winf.size());
    tb.t_wlast = em.put(sizeof(T) * wlast.size());
    std::memcpy(tb.blob.data() + tb.t_wlast, wlast.data(), sizeof(T) * wlast.size());
    tb.t_wrows = em.put(sizeof(T) * 2 * std::max<size_t>(rows, 1) * ny);
    T* wr = reinterpret_cast<T*>(tb.blob.data() + tb.t_wrows);
    for (int m = 0; m < slots; ++m) {
        for (int z = 0; z < lmax[m]; ++z) {
            T* row = wr + (size_t)(rowoff[m] + z) * ny * 2;
            for (int e = 0; e < ny; ++e) {
                for (int part = 0; part < 2; ++part) {
                    const Line<T>& ln = lines[m][(size_t)e * 2 + part];
                    row[e * 2 + part] = (z < ln.tail) ? ln.body[z] : ln.winf;
                }
            }
        }
    }
    if (ks > 0) {
        // the lower half's tables, laid out as the upper half's
        std::vector<int> boff(slots), belen((size_t)slots * ny);
        std::vector<T> bwinf((size_t)slots * ny * 2);
        size_t brows = 0;
        std::vector<int> blm(slots);
        for (int m = 0; m < slots; ++m) {
            int lm = 0;
            for (int e = 0; e < ny; ++e) {
                int el = 0;
                for (int part = 0; part < 2; ++part) {
                    const Line<T>& bl = blines[m][(size_t)e * 2 + part];
                    bwinf[((size_t)m * ny + e) * 2 + part] = bl.winf;
                    el = std::max(el, bl.tail);
                }
                belen[(size_t)m * ny + e] = el;
                lm = std::max(lm, el);
            }
            boff[m] = (int)brows;
            blm[m] = lm;
            brows += lm;
        }
        tb.t_browoff = em.put(sizeof(int) * slots);
        std::memcpy(tb.blob.data() + tb.t_browoff, boff.data(), sizeof(int) * slots);
        tb.t_belen = em.put(sizeof(int) * belen.size());
        std::memcpy(tb.blob.data() + tb.t_belen, belen.data(), sizeof(int) * belen.size());
        tb.t_bwinf = em.put(sizeof(T) * bwinf.size());
        std::memcpy(tb.blob.data() + tb.t_bwinf, bwinf.data(), sizeof(T) * bwinf.size());
        tb.t_bwrows = em.put(sizeof(T) * 2 * std::max<size_t>(brows, 1) * ny);
        T* bw = reinterpret_cast<T*>(tb.blob.data() + tb.t_bwrows);
        for (int m = 0; m < slots; ++m)
            for (int j = 0; j < blm[m]; ++j)
                for (int e = 0; e < ny; ++e)
                    for (int part = 0; part < 2; ++part) {
                        const Line<T>& bl = blines[m][(size_t)e * 2 + part];
                        bw[((size_t)(boff[m] + j) * ny + e) * 2 + part] = (j < bl.tail) ? bl.body[j] : bl.winf;
                    }
        tb.t_meet = em.put(sizeof(T) * meet.size());
        std::memcpy(tb.blob.data() + tb.t_meet, meet.data(), sizeof(T) * meet.size());
    }
    if (nseg > 0) {
        // the segmented march's tables, laid out as the top-down ones
        auto emit_seg_rows = [&](std::vector<T> SegLine<T>::*vec, T SegLine<T>::*inf, size_t* t_off, size_t* t_len,
                                 size_t* t_rows, size_t* t_inf) {
            std::vector<int> off(slots), len((size_t)slots * ny);
            std::vector<T> vinf((size_t)slots * ny * 2);
            size_t nrows = 0;
            std::vector<int> lm(slots);
            for (int m = 0; m < slots; ++m) {
                int l = 0;
                for (int e = 0; e < ny; ++e) {
                    int el = 0;
                    for (int part = 0; part < 2; ++part) {
                        const SegLine<T>& sl = slines[m][(size_t)e * 2 + part];
                        el = std::max(el, (int)(sl.*vec).size());
                        if (inf) vinf[((size_t)m * ny + e) * 2 + part] = sl.*inf;
                    }
                    len[(size_t)m * ny + e] = el;
                    l = std::max(l, el);
                }
                off[m] = (int)nrows;
                lm[m] = l;
                nrows += l;
            }
            *t_off = em.put(sizeof(int) * slots);
            std::memcpy(tb.blob.data() + *t_off, off.data(), sizeof(int) * slots);
            *t_len = em.put(sizeof(int) * len.size());
            std::memcpy(tb.blob.data() + *t_len, len.data(), sizeof(int) * len.size());
            if (t_inf) {
                *t_inf = em.put(sizeof(T) * vinf.size());
                std::memcpy(tb.blob.data() + *t_inf, vinf.data(), sizeof(T) * vinf.size());
            }
            *t_rows = em.put(sizeof(T) * 2 * std::max<size_t>(nrows, 1) * ny);
            T* rr = reinterpret_cast<T*>(tb.blob.data() + *t_rows);
            for (int m = 0; m < slots; ++m)
                for (int j = 0; j < lm[m]; ++j)
                    for (int e = 0; e < ny; ++e)
                        for (int part = 0; part < 2; ++part) {
                            const SegLine<T>& sl = slines[m][(size_t)e * 2 + part];
                            const std::vector<T>& v = sl.*vec;
                            // past its stored rows: the pivots' converged value, rho's zero
                            const T past = inf ? sl.*inf : T(0);
                            rr[((size_t)(off[m] + j) * ny + e) * 2 + part] = (j < (int)v.size()) ? v[j] : past;
                        }
        };
        emit_seg_rows(&SegLine<T>::fbody, &SegLine<T>::finf, &tb.t_frowoff, &tb.t_felen, &tb.t_fwrows, &tb.t_fwinf);
        emit_seg_rows(&SegLine<T>::rho, nullptr, &tb.t_rrowoff, &tb.t_relen, &tb.t_rrows, nullptr);
        auto emit_pair = [&](T SegLine<T>::*field, size_t* t) {
            *t = em.put(sizeof(T) * 2 * (size_t)slots * ny);
            T* v = reinterpret_cast<T*>(tb.blob.data() + *t);
            for (int m = 0; m < slots; ++m)
                for (int e = 0; e < ny; ++e)
                    for (int part = 0; part < 2; ++part)
                        v[((size_t)m * ny + e) * 2 + part] = slines[m][(size_t)e * 2 + part].*field;
        };
        emit_pair(&SegLine<T>::flast, &tb.t_flast);
        emit_pair(&SegLine<T>::rholast, &tb.t_rholast);
        tb.t_segk = em.put(sizeof(T) * 2 * 12 * (size_t)slots * ny);
        T* kk = reinterpret_cast<T*>(tb.blob.data() + tb.t_segk);
        for (int m = 0; m < slots; ++m)
            for (int e = 0; e < ny; ++e)
                for (int c = 0; c < 3; ++c)
                    for (int i = 0; i < 4; ++i)
                        for (int part = 0; part < 2; ++part)
                            kk[(((size_t)m * ny + e) * 12 + c * 4 + i) * 2 + part] =
                                (T)slines[m][(size_t)e * 2 + part].k[c][i];
    }
    // interior diagonal hz^2 lam - 2 of every z-system (PCR); padding parts get a
    // harmless non-singular value (their right-hand side is zero)
    {
        tb.t_bmid = em.put(sizeof(T) * 2 * (size_t)slots * ny);
        T* bm = reinterpret_cast<T*>(tb.blob.data() + tb.t_bmid);
        const double hz2 = p->h[2] * p->h[2];
        for (int m = 0; m < slots; ++m) {
            const bool pairslot = (p->bx != pp::BC_P) || (m == 0);
            const bool sep = (p->by == pp::BC_P) && pairslot;
            for (int e = 0; e < ny; ++e)
                for (int part = 0; part < 2; ++part) {
                    int kx, ky;
                    if (sep && e != 0 && 2 * e != ny) {
                        kx = kx_of(m, e < ny - e ? 0 : 1);
                        ky = e;
                    } else {
                        kx = kx_of(m, part);
                        ky = (p->by == pp::BC_D) ? ny - 1 - e : e;
                    }
                    bm[((size_t)m * ny + e) * 2 + part] = (kx < 0) ? T(-3) : (T)(-2.0 + hz2 * (lamx[kx] + lamy[ky]));
                }
        }
    }
    if (p->bz0 != pp::BC_P) return;
    // periodic z: Sherman-Morrison rows (alpha, qp) per slot, and per-entry scalars
    auto emit_rows = [&](std::vector<T> Line<T>::*vec, size_t* t_off, size_t* t_len, size_t* t_rows, size_t* t_elen) {
        std::vector<int> off(slots), len(slots), elen((size_t)slots * ny);
        for (int m = 0; m < slots; ++m)
            for (int e = 0; e < ny; ++e)
                elen[(size_t)m * ny + e] = (int)std::max((lines[m][(size_t)e * 2].*vec).size(),
                                                         (lines[m][(size_t)e * 2 + 1].*vec).size());
        *t_elen = em.put(sizeof(int) * elen.size());
        std::memcpy(tb.blob.data() + *t_elen, elen.data(), sizeof(int) * elen.size());
        size_t nrows = 0;
        for (int m = 0; m < slots; ++m) {
            int L = 0;
            for (const Line<T>& ln : lines[m]) L = std::max(L, (int)(ln.*vec).size());
            off[m] = (int)nrows;
            len[m] = L;
            nrows += L;
        }
        *t_off = em.put(sizeof(int) * slots);
        std::memcpy(tb.blob.data() + *t_off, off.data(), sizeof(int) * slots);
        *t_len = em.put(sizeof(int) * slots);
        std::memcpy(tb.blob.data() + *t_len, len.data(), sizeof(int) * slots);
        *t_rows = em.put(sizeof(T) * 2 * std::max<size_t>(nrows, 1) * ny);
        T* rr = reinterpret_cast<T*>(tb.blob.data() + *t_rows);
        for (int m = 0; m < slots; ++m)
            for (int z = 0; z < len[m]; ++z)
                for (int e = 0; e < ny; ++e)
                    for (int part = 0; part < 2; ++part) {
                        const std::vector<T>& v = lines[m][(size_t)e * 2 + part].*vec;
                        rr[((size_t)(off[m] + z) * ny + e) * 2 + part] = (z < (int)v.size()) ? v[z] : T(0);
                    }
    };
    emit_rows(&Line<T>::alpha, &tb.t_aoff, &tb.t_alen, &tb.t_arows, &tb.t_aelen);
    emit_rows(&Line<T>::qp, &tb.t_qoff, &tb.t_qlen, &tb.t_qrows, &tb.t_qelen);
    auto emit_scalar = [&](T Line<T>::*field, size_t* t) {
        *t = em.put(sizeof(T) * 2 * (size_t)slots * ny);
        T* v = reinterpret_cast<T*>(tb.blob.data() + *t);
        for (int m = 0; m < slots; ++m)
            for (int e = 0; e < ny; ++e)
                for (int part = 0; part < 2; ++part)
                    v[((size_t)m * ny + e) * 2 + part] = lines[m][(size_t)e * 2 + part].*field;
    };
    emit_scalar(&Line<T>::qlast, &tb.t_qlast);
    emit_scalar(&Line<T>::inv_den, &tb.t_invden);
    emit_scalar(&Line<T>::inv_gamma, &tb.t_invgam);
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Spectral array layout.  z-major ([b][z][slot][y]): the workgroups of the z
// march, one per slot, advance through z together, so at any moment they touch
// one contiguous stretch of the array rather than one line in each of a few
// hundred columns a power of two apart; the x kernels write and read whole
// z planes either way.
#ifndef PP_SPECTRAL_ZMAJOR
#define PP_SPECTRAL_ZMAJOR 1
#endif
void spectral_strides(pp_plan p, long* sstride, long* zstride) {
    if (PP_SPECTRAL_ZMAJOR) {
        *sstride = p->ny;
        *zstride = (long)p->slots * p->ny;
    } else {
        *sstride = (long)p->nz * p->ny;
        *zstride = p->ny;
    }
}

// Refined solve: the spectral slots of the smallest x wavenumbers, whose z
// systems are the least well conditioned, are kept in double by the forward x
// transform and solved in double by the mixed z march.  Float rounding of
// their spectra (which mix every y wavenumber) and of their y transforms and
// recurrences is amplified by up to |lam_max / lam| in the solution; in the
// other slots |lam_x| alone bounds that factor.  Periodic and cosine x hold
// those wavenumbers in the first slots, sine x (columns stored reversed) in
// the last.  Only where the mixed march exists (otherwise the refinement
// simply takes more corrections).
//
// The stop rule may then take the first correction as the contraction factor
// (fast_stop) when the float slots amplify rounding by at most kFastStopBound:
// the largest eigenvalue magnitude over the smallest |lam_x| of a float slot
// (measured: a bound of 310 at 512^3 and 415 on 8 x 16 x 1024 give corrections
// that contract by ~3e-7; with no double slots, 13 x 1024 x 6 contracted by
// only 4.5e-4).
constexpr int kMixedSlots = 16;
constexpr double kFastStopBound = 1000.0;
void set_mixed_slots(pp_plan p) {
    p->nlo = 0;
    p->lo0 = 0;
    p->fast_stop = false;
    if (!pp::mixed_march_supported(p->ny, p->zsolver)) return;
    p->nlo = std::min(p->slots, kMixedSlots);
    p->lo0 = (p->bx == pp::BC_D) ? p->slots - p->nlo : 0;
    const int nx = p->nx;
    double lmax = 0.0;
    for (int d = 0; d < 3; ++d) lmax += 4.0 / (p->h[d] * p->h[d]);
    double lmin = 0.0;   // smallest |lam_x| of a float slot (0: none)
    for (int m = 0; m < p->slots; ++m) {
        if (m >= p->lo0 && m < p->lo0 + p->nlo) continue;
        for (int part = 0; part < 2; ++part) {
            int kx;
            if (p->bx == pp::BC_P) kx = (m == 0) ? (part ? nx / 2 : 0) : m;
            else kx = 2 * m + part;   // DCT index; DST columns hold index nx-1-k, covered by the loop
            if (kx >= nx) continue;
            const int k = (p->bx == pp::BC_D) ? nx - 1 - kx : kx;
            const double l = std::fabs(eigenvalue(p->bx, k, nx, p->h[0]));
            if (lmin == 0.0 || l < lmin) lmin = l;
        }
    }
    p->fast_stop = (lmin == 0.0) ? true : (lmax / lmin <= kFastStopBound);
}

template <typename T> pp::XArgs<T> make_xargs(pp_plan p, unsigned char* ws, int set = 0) {
    const Tables& tb = p->tb[set];
    pp::XArgs<T> a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.slots = p->slots;
    a.bx = p->bx;
    a.ty = p->ty;
    a.ldl = p->ldl;
    spectral_strides(p, &a.sstride, &a.zstride);
    a.fx = p->fx;
    unsigned char* t = ws + p->o_tab[set];
    a.twx = reinterpret_cast<const cplx<T>*>(t + tb.t_twx);
    a.mkx = reinterpret_cast<const cplx<T>*>(t + tb.t_mkx);
    a.lo0 = 0;
    a.nlo = 0;
    a.slo = nullptr;
    return a;
}

// Per-batch arrays after the fixed scalars: [0, B) mean of the right-hand side
// of the current solve, [B, 2B) mean of the zero-mode solution line, [2B, 3B)
// gauge shift of the refinement loop, [3B, 4B) mean of the source f.
template <typename T>
pp::MidArgs<T> make_midargs(pp_plan p, unsigned char* ws, bool project, bool demean, int set = 0) {
    const Tables& tb = p->tb[set];
    pp::MidArgs<T> a{};
    a.ny = p->ny;
    a.nz = p->nz;
    a.slots = p->slots;
    a.bx = p->bx;
    a.by = p->by;
    a.ldy = p->ldy;
    a.zb = p->zb;
    spectral_strides(p, &a.sstride, &a.zstride);
    a.singular = p->singular ? 1 : 0;
    a.project = project ? 1 : 0;
    a.demean = demean ? 1 : 0;
    a.scale = (T)(p->h[2] * p->h[2] / ((double)p->nx * (double)p->ny));
    a.hz2 = p->h[2] * p->h[2];
    a.fy = p->fy;
    unsigned char* t = ws + p->o_tab[set];
    a.twy = reinterpret_cast<const cplx<T>*>(t + tb.t_twy);
    a.mky = reinterpret_cast<const cplx<T>*>(t + tb.t_mky);
    a.rowoff = reinterpret_cast<const int*>(t + tb.t_rowoff);
    a.lmax = reinterpret_cast<const int*>(t + tb.t_lmax);
    a.elen = reinterpret_cast<const int*>(t + tb.t_elen);
    a.wrows = reinterpret_cast<const cplx<T>*>(t + tb.t_wrows);
    a.winf = reinterpret_cast<const cplx<T>*>(t + tb.t_winf);
    a.wlast = reinterpret_cast<const cplx<T>*>(t + tb.t_wlast);
    // the split march where the columns alone would leave half the compute
    // units or more without a workgroup
    // automatic, by columns (slots x batch) per compute unit, as measured:
    // double at most 1/2 (one workgroup per CU either way: 256^3 with 128
    // columns 0.31 -> 0.18 ms; 192 or 256 columns 2-5% slower split); float at
    // most 2 (the halves run two per CU: 512^3 0.53 -> 0.44 ms, 1024^2 x 512
    // 2.50 -> 2.36 ms; 768 columns 11% slower); the refined solve's mixed
    // march at most 4 (768 columns of 384^3 x 4: 1.61 -> 1.30 ms).
    // Double on lines up to 512, beyond one column per CU: each workgroup's
    // march is latency-bound, so the whole march takes ceil(c / CUs) rounds
    // of one column's time T however full its last round is, and the split
    // two launches of ceil(2c / CUs) rounds of about 0.26 T; split where
    // that is shorter (384^3 DD DD DD: 576 columns 2.02 -> 1.75 ms, 1152
    // 3.37 -> 3.05; 768 and 960 columns whole, 2.05 and 2.71 ms)
    a.zsplit = 0;
    const long long cols = (long long)p->slots * p->batch, cus = pp::device_cus();
    long long lim = p->dtype == PP_F64 ? cus / 2 : (p->dtype == PP_F32 ? 2 * cus : 4 * cus);
    if (p->dtype == PP_F64 && p->ny <= 512 && cols > cus) {
        const long long whole = (cols + cus - 1) / cus, halves = (2 * cols + cus - 1) / cus;
        if (13 * halves < 25 * whole) lim = cols;
    }
    // the amplification bound holds double plans to the single march's
    // accuracy; float rounding (6e-8) dominates the two-way split's meeting
    // rows (512^3 periodic x, y: 1.97e-6 split, 1.81e-6 whole, from the f64
    // solve) but not the segmented march's (1023 x 16 x 16: 3.7e-5 vs 1.5e-6)
    const bool tame = p->split_gmax <= kSplitGMax;
    const bool split = p->zsplit_mode == PP_ZSPLIT_ON ||
                       (p->zsplit_mode == PP_ZSPLIT_AUTO && cols <= lim && (p->dtype != PP_F64 || tame));
    if (p->zsplit > 0 && p->zsolver == 0 && split) {
        a.zsplit = p->zsplit;
        a.browoff = reinterpret_cast<const int*>(t + tb.t_browoff);
        a.belen = reinterpret_cast<const int*>(t + tb.t_belen);
        a.bwinf = reinterpret_cast<const cplx<T>*>(t + tb.t_bwinf);
        a.bwrows = reinterpret_cast<const cplx<T>*>(t + tb.t_bwrows);
        a.meet = reinterpret_cast<const cplx<T>*>(t + tb.t_meet);
        a.zbuf = reinterpret_cast<cplx<T>*>(ws + p->o_zb[set]);
    }
    // the segmented march where the plan has one (f64 and f32 plans with few
    // columns), unless a layout is forced (also where the columns alone would
    // not split: double lines up to 256 with 129-256 columns, 256^3 DD NN NN
    // x 2: 0.351 -> 0.293 ms; 384 x 256 x 256: 0.330 -> 0.231 ms)
    a.zsegs = 0;
    if (p->zsegs > 0 && p->zsolver == 0 &&
        (p->zsplit_mode == PP_ZSPLIT_SEG || (p->zsplit_mode == PP_ZSPLIT_AUTO && tame))) {
        a.zsplit = 0;
        a.zsegs = p->zsegs;
        a.zseglen = p->zseglen;
        a.frowoff = reinterpret_cast<const int*>(t + tb.t_frowoff);
        a.felen = reinterpret_cast<const int*>(t + tb.t_felen);
        a.fwrows = reinterpret_cast<const cplx<T>*>(t + tb.t_fwrows);
        a.fwinf = reinterpret_cast<const cplx<T>*>(t + tb.t_fwinf);
        a.flast = reinterpret_cast<const cplx<T>*>(t + tb.t_flast);
        a.rrowoff = reinterpret_cast<const int*>(t + tb.t_rrowoff);
        a.relen = reinterpret_cast<const int*>(t + tb.t_relen);
        a.rrows = reinterpret_cast<const cplx<T>*>(t + tb.t_rrows);
        a.rholast = reinterpret_cast<const cplx<T>*>(t + tb.t_rholast);
        a.segk = reinterpret_cast<const cplx<T>*>(t + tb.t_segk);
        const size_t unit = (size_t)p->batch * p->slots * p->zsegs * p->ny;
        a.segg = reinterpret_cast<cplx<T>*>(ws + p->o_seg);
        a.seglr = a.segg + 2 * unit;
    }
    a.zsolver = p->zsolver;
    a.bz0 = p->bz0;
    a.bz1 = p->bz1;
    a.bmid = reinterpret_cast<const cplx<T>*>(t + tb.t_bmid);
    a.zper = (p->bz0 == pp::BC_P) ? 1 : 0;
    if (a.zper) {
        a.aoff = reinterpret_cast<const int*>(t + tb.t_aoff);
        a.alen = reinterpret_cast<const int*>(t + tb.t_alen);
        a.aelen = reinterpret_cast<const int*>(t + tb.t_aelen);
        a.qelen = reinterpret_cast<const int*>(t + tb.t_qelen);
        a.arows = reinterpret_cast<const cplx<T>*>(t + tb.t_arows);
        a.qoff = reinterpret_cast<const int*>(t + tb.t_qoff);
        a.qlen = reinterpret_cast<const int*>(t + tb.t_qlen);
        a.qrows = reinterpret_cast<const cplx<T>*>(t + tb.t_qrows);
        a.qlast = reinterpret_cast<const cplx<T>*>(t + tb.t_qlast);
        a.inv_den = reinterpret_cast<const cplx<T>*>(t + tb.t_invden);
        a.inv_gamma = reinterpret_cast<const cplx<T>*>(t + tb.t_invgam);
    }
    double* sc = reinterpret_cast<double*>(ws + p->o_scalars);
    a.mu = sc + pp::SC_COUNT + 3 * p->batch;
    a.cmean = sc + pp::SC_COUNT + p->batch;
    return a;
}

// Record a timing event before a launch of kernel group `group` (-1: end of a
// sequence).  No-op unless timing is on.
pp_status mark(pp_plan p, hipStream_t s, int group) {
    if (!p->timing) return PP_OK;
    const size_t idx = p->marks.size();
    if (idx >= p->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return PP_ERR_HIP;
        p->ev_pool.push_back(e);
    }
    if (hipEventRecord(p->ev_pool[idx], s) != hipSuccess) return PP_ERR_HIP;
    p->marks.emplace_back((int)idx, group);
    return PP_OK;
}

// Fold the recorded marks into the per-group accumulators.
pp_status collect(pp_plan p) {
    if (p->marks.empty()) return PP_OK;
    if (hipEventSynchronize(p->ev_pool[p->marks.back().first]) != hipSuccess) return PP_ERR_HIP;
    for (size_t i = 0; i + 1 < p->marks.size(); ++i) {
        const int g = p->marks[i].second;
        if (g < 0) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev_pool[p->marks[i].first], p->ev_pool[p->marks[i + 1].first]) != hipSuccess)
            return PP_ERR_HIP;
        p->kms[g] += ms;
        p->kcount[g] += 1;
    }
    p->marks.clear();
    return PP_OK;
}

#define PP_HIP(call)                          \
    do {                                      \
        if ((call) != hipSuccess) return PP_ERR_HIP; \
    } while (0)

// Partial records per batch entry written by an x kernel on this device
// (<= p->nper, which sizes the partial region of the workspace); paired: the
// inverse kernel with float spectra, which runs half the workgroups.
int x_records(pp_plan p, bool paired) {
    return pp::x_launch_grid(pp::x_blocks(p->ny, p->ty, p->nz, p->batch), paired) * pp::kXWaves;
}

template <typename T, typename Tio>
pp_status run_plain(pp_plan p, const Tio* f, Tio* u, unsigned char* ws, hipStream_t s, bool project, bool demean,
                    const pp::FaceArgs<Tio>* faces) {
    pp::XArgs<T> xa = make_xargs<T>(p, ws);
    pp::MidArgs<T> ma = make_midargs<T>(p, ws, project, demean);
    xa.zends = ma.zsplit > 0;
    double* sc = reinterpret_cast<double*>(ws + p->o_scalars);
    double* partial = reinterpret_cast<double*>(ws + p->o_partial);
    cplx<T>* S = reinterpret_cast<cplx<T>*>(ws + p->o_S);
    const double npts = (double)p->nx * p->ny * p->nz;
    pp_status st;
    if ((st = mark(p, s, 0)) != PP_OK) return st;
    PP_HIP((pp::launch_xfwd<T, Tio, T>(f, S, partial, xa, p->batch, faces, s)));
    if ((st = mark(p, s, 3)) != PP_OK) return st;
    PP_HIP(pp::launch_finalize_xfwd(partial, x_records(p, false), p->batch, npts,
                                    sc + pp::SC_COUNT + 3 * p->batch, sc + pp::SC_MAXF, s));
    if ((st = mark(p, s, 1)) != PP_OK) return st;
    PP_HIP(pp::launch_mid<T>(S, ma, p->batch, s));
    if ((st = mark(p, s, 2)) != PP_OK) return st;
    PP_HIP((pp::launch_xinv<T, Tio>(S, u, xa, p->batch, sc + pp::SC_COUNT + p->batch, s)));
    return mark(p, s, -1);
}

// z stage of a refined solve: the mixed march where it exists (the double
// slots from their double spectra), else the float march.
pp_status refined_mid(pp_plan p, unsigned char* ws, const pp::MidArgs<float>& ma, const pp::MidArgs<double>& ma64,
                      hipStream_t s) {
    cplx<float>* S = reinterpret_cast<cplx<float>*>(ws + p->o_S);
    if (p->nlo > 0) {
        const cplx<double>* Slo = reinterpret_cast<const cplx<double>*>(ws + p->o_lo);
        PP_HIP(pp::launch_mid_mixed(Slo, S, ma64, ma, p->lo0, p->nlo, p->batch, s));
    } else {
        PP_HIP(pp::launch_mid<float>(S, ma, p->batch, s));
    }
    return PP_OK;
}

// FP32 solves wrapped in iterative refinement with an FP64 residual and update.
// Every solve transforms along x in double arithmetic and keeps the spectra of
// the slots of the smallest x wavenumbers in double (set_mixed_slots); the
// rest of the solve runs in float.  The first solution u0 is kept in float (it
// is a float solve's result); the first correction reads it and writes u in
// double; any further correction updates u in place.
pp_status run_refined(pp_plan p, const double* f, double* u, unsigned char* ws, hipStream_t s, bool project,
                      bool demean, const pp::FaceArgs<double>* faces) {
    pp::XArgs<double> xa64 = make_xargs<double>(p, ws, 1);   // forward: double arithmetic, split store
    xa64.lo0 = p->lo0;
    xa64.nlo = p->nlo;
    xa64.slo = reinterpret_cast<cplx<double>*>(ws + p->o_lo);
    pp::XArgs<float> xa = make_xargs<float>(p, ws, 0);       // inverse: float
    pp::MidArgs<float> ma = make_midargs<float>(p, ws, project, demean, 0);
    pp::MidArgs<double> ma64 = make_midargs<double>(p, ws, project, demean, 1);
    xa.zends = ma.zsplit > 0;
    double* sc = reinterpret_cast<double*>(ws + p->o_scalars);
    double* partial = reinterpret_cast<double*>(ws + p->o_partial);
    cplx<float>* S = reinterpret_cast<cplx<float>*>(ws + p->o_S);
    float* u0 = reinterpret_cast<float*>(ws + p->o_u0);   // first solution
    // the residual of the first correction is formed inside the forward x
    // transform (rows up to 512); otherwise it is stored, in double: a float
    // residual rounds the part the first solution's float rounding puts into it,
    // which is large where one direction is much finer than the others, and the
    // float solve of that rounding limits the correction (to ~1e-5 of its size
    // on 8 x 8 x 512 and 8 x 16 x 1024 grids, against ~3e-7 here).  Later
    // corrections (rare) form a float residual in u0's array.
    const bool fused = pp::res_fused_supported(p->nx);
    double* r64 = reinterpret_cast<double*>(ws + p->o_r);
    float* r32 = u0;
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const double npts = (double)n;
    // gauge region whose mean is held fixed across corrections:
    // 1 = volume (zero-mean gauge), 2 = plane z = 0 (pinned gauge)
    int region = 0;
    double nregion = 0.0;
    if (p->singular) {
        region = demean ? 1 : 2;
        nregion = demean ? npts : (double)p->nx * p->ny;
    }
    pp::ResidualArgs ra{};
    ra.nx = p->nx;
    ra.ny = p->ny;
    ra.nz = p->nz;
    ra.batch = p->batch;
    for (int i = 0; i < 6; ++i) ra.bc[i] = bc_code(p->bc[i]);
    ra.proj = p->singular ? (project ? 1 : 2) : 0;
    ra.ihx2 = 1.0 / (p->h[0] * p->h[0]);
    ra.ihy2 = 1.0 / (p->h[1] * p->h[1]);
    ra.ihz2 = 1.0 / (p->h[2] * p->h[2]);
    if (faces) {
        ra.faces = *faces;
        ra.has_faces = 1;
    }
    const bool keep_u0 = p->ir_max > 0;   // with no correction the float solve goes straight to u

    pp_status st;
    if ((st = mark(p, s, 3)) != PP_OK) return st;
    PP_HIP(pp::launch_ir_init(sc, p->batch, s));
    if ((st = mark(p, s, 0)) != PP_OK) return st;
    PP_HIP((pp::launch_xfwd<double, double, float>(f, S, partial, xa64, p->batch, faces, s)));
    if ((st = mark(p, s, 3)) != PP_OK) return st;
    PP_HIP(pp::launch_finalize_xfwd(partial, x_records(p, false), p->batch, npts, sc + pp::SC_COUNT + 3 * p->batch,
                                    sc + pp::SC_MAXF, s));
    if ((st = mark(p, s, 1)) != PP_OK) return st;
    if ((st = refined_mid(p, ws, ma, ma64, s)) != PP_OK) return st;
    ma.mu = sc + pp::SC_COUNT;   // corrections project their own right-hand side
    ma64.mu = sc + pp::SC_COUNT;
    if ((st = mark(p, s, 2)) != PP_OK) return st;
    if (keep_u0) PP_HIP(pp::launch_xinv_first(S, u0, xa, p->batch, sc, region, partial, s));
    else PP_HIP(pp::launch_xinv_update(S, u, nullptr, xa, p->batch, sc, region, partial, pp::XINV_FIRST, s));
    if ((st = mark(p, s, 3)) != PP_OK) return st;
    PP_HIP(pp::launch_finalize_update(partial, x_records(p, true), p->batch, nregion, sc, 1, s));
    if ((st = mark(p, s, -1)) != PP_OK) return st;
    p->last_iters = 0;
    p->last_rel = 1.0;
    for (int it = 1; it <= p->ir_max; ++it) {
        if (fused && it == 1) {
            pp::XArgs<double> xr = xa64;
            xr.u0 = u0;
            xr.sc = sc;
            for (int i = 0; i < 6; ++i) xr.fbc[i] = ra.bc[i];
            xr.proj = ra.proj;
            xr.ihx2 = ra.ihx2;
            xr.ihy2 = ra.ihy2;
            xr.ihz2 = ra.ihz2;
            if ((st = mark(p, s, 0)) != PP_OK) return st;
            PP_HIP(pp::launch_xfwd_res(f, S, partial, xr, p->batch, faces, s));
        } else if (fused) {
            if ((st = mark(p, s, 3)) != PP_OK) return st;
            PP_HIP((pp::launch_residual<double, float>(f, u, r32, ra, sc, s)));
            if ((st = mark(p, s, 0)) != PP_OK) return st;
            PP_HIP((pp::launch_xfwd<double, float, float>(r32, S, partial, xa64, p->batch, nullptr, s)));
        } else {
            if ((st = mark(p, s, 3)) != PP_OK) return st;
            if (it == 1) PP_HIP((pp::launch_residual<float, double>(f, u0, r64, ra, sc, s)));
            else PP_HIP((pp::launch_residual<double, double>(f, u, r64, ra, sc, s)));
            if ((st = mark(p, s, 0)) != PP_OK) return st;
            PP_HIP((pp::launch_xfwd<double, double, float>(r64, S, partial, xa64, p->batch, nullptr, s)));
        }
        if ((st = mark(p, s, 3)) != PP_OK) return st;
        PP_HIP(pp::launch_finalize_xfwd(partial, x_records(p, false), p->batch, npts, sc + pp::SC_COUNT, nullptr, s));
        if ((st = mark(p, s, 1)) != PP_OK) return st;
        if ((st = refined_mid(p, ws, ma, ma64, s)) != PP_OK) return st;
        if ((st = mark(p, s, 2)) != PP_OK) return st;
        PP_HIP(pp::launch_xinv_update(S, u, it == 1 ? u0 : nullptr, xa, p->batch, sc, region, partial,
                                      pp::XINV_UPDATE, s));
        if ((st = mark(p, s, 3)) != PP_OK) return st;
        PP_HIP(pp::launch_finalize_update(partial, x_records(p, true), p->batch, nregion, sc, 0, s));
        if ((st = mark(p, s, -1)) != PP_OK) return st;
        double h[8];
        PP_HIP(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, s));
        PP_HIP(hipStreamSynchronize(s));
        p->last_iters = it;
        const double maxf = h[pp::SC_MAXF], rel = h[pp::SC_REL], relprev = h[pp::SC_RELPREV];
        p->last_rel = rel;
        if ((st = collect(p)) != PP_OK) return st;
        if (!std::isfinite(maxf) || !std::isfinite(rel)) return PP_ERR_NONFINITE;
        // estimated error after this correction: the next correction, the size
        // of this one times the contraction factor.  After two corrections the
        // factor is their ratio; after the first, with fast_stop, it is the
        // first correction itself, the relative error of the first solve, which
        // the correction's own solve (the same float solve) is taken to repeat;
        // otherwise 1 (the first correction must itself be below the tolerance).
        double rho = 1.0;
        if (it >= 2 && relprev > 0.0) rho = std::min(1.0, rel / relprev);
        else if (it == 1 && p->fast_stop) rho = std::min(1.0, rel);
        if (rel == 0.0 || rel * rho <= p->ir_tol) return PP_OK;
    }
    return PP_ERR_NOT_CONVERGED;
}

// Face-value block of a non-homogeneous solve.  Absent faces read from f with a
// zero coefficient, so the kernels load every face unconditionally (f is at
// least as large as any face array).
template <typename Tin> pp::FaceArgs<Tin> face_args(pp_plan p, const void* f, const void* const* faces) {
    pp::FaceArgs<Tin> fa{};
    for (int i = 0; i < 6; ++i) {
        const double hd = p->h[i / 2];
        if (faces[i]) {
            fa.g[i] = reinterpret_cast<const Tin*>(faces[i]);
            fa.c[i] = (p->bc[i] == 'D') ? 2.0 / (hd * hd) : 1.0 / hd;
        } else {
            fa.g[i] = reinterpret_cast<const Tin*>(f);
            fa.c[i] = 0.0;
        }
    }
    return fa;
}

// Elements of face i per batch entry: x faces nz*ny, y faces nz*nx, z faces ny*nx.
size_t face_elems(pp_plan p, int i) {
    const int d = i / 2;
    if (d == 0) return (size_t)p->nz * p->ny;
    if (d == 1) return (size_t)p->nz * p->nx;
    return (size_t)p->ny * p->nx;
}

pp_status dispatch(pp_plan p, const void* f, void* u, void* workspace, void* stream, bool adjoint,
                   const void* const* faces = nullptr) {
    if (!p || !f || !u) return PP_ERR_ARG;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return PP_ERR_WORKSPACE;
    const size_t n = (size_t)p->nx * p->ny * p->nz * p->batch;
    const size_t io = (p->dtype == PP_F32) ? sizeof(float) : sizeof(double);
    if (((uintptr_t)f % io) != 0 || ((uintptr_t)u % io) != 0) return PP_ERR_ARG;
    if (overlap(f, n * io, u, n * io) || overlap(u, n * io, workspace, p->ws_bytes) ||
        overlap(f, n * io, workspace, p->ws_bytes))
        return PP_ERR_ALIAS;
    bool any_face = false;
    if (faces) {
        for (int i = 0; i < 6; ++i) {
            if (!faces[i]) continue;
            if (p->bc[i] == 'P') return PP_ERR_ARG;   // periodic faces carry no values
            if (((uintptr_t)faces[i] % io) != 0) return PP_ERR_ARG;
            const size_t nb = face_elems(p, i) * p->batch * io;
            if (overlap(faces[i], nb, u, n * io) || overlap(faces[i], nb, workspace, p->ws_bytes))
                return PP_ERR_ALIAS;
            any_face = true;
        }
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
    if (!tables_present(p, workspace)) {
        for (int i = 0; i < p->ntab; ++i)
            PP_HIP(hipMemcpyAsync(ws + p->o_tab[i], p->tb[i].blob.data(), p->tb[i].blob.size(), hipMemcpyHostToDevice,
                                  s));
        tables_uploaded(p, workspace);
    }
    // zero-mode treatment; the adjoint trades projection and mean shift
    bool project, demean;
    if (!adjoint) {
        project = p->gauge != PP_GAUGE_PIN_RAW;
        demean = p->gauge == PP_GAUGE_MEAN;
    } else {
        project = p->gauge == PP_GAUGE_MEAN;
        demean = p->gauge != PP_GAUGE_PIN_RAW;
    }
    if (p->marks.size() > 4096) {
        const pp_status st = collect(p);
        if (st != PP_OK) return st;
    }
    p->last_ws = workspace;
    p->last_stream = s;
    p->last_iters = 0;
    p->last_rel = 0.0;
    p->last_projected = p->singular && project;
    switch (p->dtype) {
        case PP_F64: {
            const pp::FaceArgs<double> fa = any_face ? face_args<double>(p, f, faces) : pp::FaceArgs<double>{};
            return run_plain<double, double>(p, (const double*)f, (double*)u, ws, s, project, demean,
                                             any_face ? &fa : nullptr);
        }
        case PP_F32: {
            const pp::FaceArgs<float> fa = any_face ? face_args<float>(p, f, faces) : pp::FaceArgs<float>{};
            return run_plain<float, float>(p, (const float*)f, (float*)u, ws, s, project, demean,
                                           any_face ? &fa : nullptr);
        }
        case PP_F32_REFINED: {
            const pp::FaceArgs<double> fa = any_face ? face_args<double>(p, f, faces) : pp::FaceArgs<double>{};
            return run_refined(p, (const double*)f, (double*)u, ws, s, project, demean, any_face ? &fa : nullptr);
        }
    }
    return PP_ERR_ARG;
}

}  // namespace

extern "C" {

pp_status pp_plan_create(int nx, int ny, int nz, const char bc[6], const double h[3], pp_dtype dtype, int batch,
                         pp_plan* out) {
    if (!out) return PP_ERR_ARG;
    *out = nullptr;
    if (!bc || !h) return PP_ERR_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || batch < 1) return PP_ERR_ARG;
    if (dtype != PP_F64 && dtype != PP_F32 && dtype != PP_F32_REFINED) return PP_ERR_ARG;
    for (int d = 0; d < 3; ++d)
        if (!(h[d] > 0.0) || !std::isfinite(h[d])) return PP_ERR_ARG;
    int code[6];
    for (int i = 0; i < 6; ++i) {
        code[i] = bc_code(bc[i]);
        if (code[i] < 0) return PP_ERR_BC;
    }
    if (code[0] != code[1] || code[2] != code[3]) return PP_ERR_BC;
    if ((code[4] == pp::BC_P) != (code[5] == pp::BC_P)) return PP_ERR_BC;   // periodic z needs both faces
    if (code[4] == pp::BC_P && nz < 3) return PP_ERR_SIZE;                     // Sherman-Morrison splitting
    if (!factor23(nx) || !factor23(ny)) return PP_ERR_SIZE;
    if (nx > pp::kMaxLine || ny > pp::kMaxLine || ny > pp::kZThreads * pp::kZOwned) return PP_ERR_SIZE;
    if ((long long)nz * batch > 65535) return PP_ERR_SIZE;

    pp_plan p = new (std::nothrow) pp_plan_s;
    if (!p) return PP_ERR_ARG;
    {
        std::lock_guard<std::mutex> lock(g_ws_mu);
        p->serial = g_next_serial++;
    }
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->batch = batch;
    std::memcpy(p->bc, bc, 6);
    std::memcpy(p->h, h, sizeof(double) * 3);
    p->dtype = dtype;
    p->bx = code[0];
    p->by = code[2];
    p->bz0 = code[4];
    p->bz1 = code[5];
    p->singular = (p->bx != pp::BC_D) && (p->by != pp::BC_D) &&
                  ((p->bz0 == pp::BC_N && p->bz1 == pp::BC_N) || p->bz0 == pp::BC_P);
    p->slots = (nx + 1) / 2;
    const bool f64 = (dtype == PP_F64);
    p->elem = f64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
    p->fx = radix_plan(nx);
    p->fy = radix_plan(ny);
    p->ldl = pp::padded_len(nx);
    p->ldy = pp::padded_len(ny);
    // row pairs (lines) per x workgroup: each wavefront transforms lpw whole lines
    // (64 * rmax >= lpw * nx values); capped by the rows present
    int lines;
    {
        const int epl = (nx + 63) / 64;
        // (rows of 256: one line per wavefront, the exact-count form with four values per lane)
        const int lpw = (nx == 256) ? 1 : std::max(1, pp::xdir_rmax(nx) / epl);
        lines = std::min(pp::kXWaves * lpw, (ny + 1) / 2);
        // the inverse gathers slots * lines (slot, row pair) values, rmax/2 per thread
        while (lines > 1 && (size_t)((nx + 1) / 2) * lines > (size_t)pp::kXThreads * (pp::xdir_rmax(nx) / 2)) --lines;
        // LDS: the lines plus two twiddle tables of nx; fewer lines to keep two
        // workgroups per CU, and a single line may use the whole LDS
        // (the refined solve's forward x transform works in double)
        const size_t xelem = (dtype == PP_F32) ? sizeof(cplx<float>) : sizeof(cplx<double>);
        auto xlds = [&](int l) { return ((size_t)l * pp::padded_len(nx) + 2 * (size_t)nx) * xelem; };
        const int lines_all = lines;
        while (lines > 1 && xlds(lines) > (size_t)pp::kXLdsBytes) --lines;
        // except for the exact-count shape (one line of 64 rmax values per
        // wavefront, kXWaves lines): kept at one workgroup per CU when its LDS
        // allows (double rows of 1024), since the general form is slower still
        if (lines_all == pp::kXWaves && lpw == 1 && nx == 64 * pp::xdir_rmax(nx) && xlds(lines_all) <= (size_t)pp::kXLdsMax)
            lines = lines_all;
        if (xlds(lines) > (size_t)pp::kXLdsMax) lines = 0;
    }
    // z planes per chunk: each wavefront of the z march transforms whole planes,
    // ppw = rmax / ceil(ny/64) of them per chunk; the LDS holds the chunk and the twiddles
    {
        const int nw = pp::kZThreads / 64;
        const int epl = (ny + 63) / 64;
        const int ppw = pp::zmarch_rmax(ny) / epl;
        const int ldy = pp::padded_len(ny);
        const int zb_lds = (int)((pp::kZLdsBytes / p->elem - (size_t)ny) / (size_t)ldy);
        p->zb = std::min({nw * ppw, nz, zb_lds});
    }
    if (lines < 1 || p->zb < 1) {
        delete p;
        return PP_ERR_SIZE;
    }
    p->ty = 2 * lines;
    // partial records per batch entry: one per (workgroup, wavefront) of the persistent
    // x kernels, whose grid never exceeds the row blocks of all batch entries
    p->nper = (size_t)((ny + p->ty - 1) / p->ty) * nz * batch * pp::kXWaves;
    // split march: the meeting point on a chunk boundary near the middle (the
    // refined solve's march has the float march's chunks)
    {
        const int kz = pp::zpipe_planes(ny, f64);
        const int nch = kz > 0 ? (nz + kz - 1) / kz : 0;
        if (p->bz0 != pp::BC_P && kz > 0 && nz >= 2 * kz) p->zsplit = kz * ((nch + 1) / 2);
        // segmented march (f64 and f32 plans): enough segments per column to
        // give MI355X's 256 CUs a workgroup each, of whole chunks, at least two
        // chunks long; only where that means three segments or more
        if (p->zsplit > 0 && dtype != PP_F32_REFINED) {
            const long long cols = (long long)p->slots * batch;
            const long long target =
                ny <= 256 ? (f64 ? kSegTargetNarrowF64 : kSegTargetNarrowF32) : kSegTargetColumns;
            int nseg = (int)std::min<long long>(kMaxSegments, target / std::max<long long>(cols, 1));
            if (nseg >= 3) {
                int len = (nz + nseg - 1) / nseg;
                len = std::max(2 * kz, (len + kz - 1) / kz * kz);
                nseg = (nz + len - 1) / len;
                if (nseg >= 3) {
                    p->zsegs = nseg;
                    p->zseglen = len;
                }
            }
        }
    }
    if (f64) build_tables<double>(p, p->tb[0]);
    else build_tables<float>(p, p->tb[0]);
    if (dtype == PP_F32_REFINED) {
        build_tables<double>(p, p->tb[1]);
        p->ntab = 2;
        set_mixed_slots(p);
    }

    const size_t n = (size_t)nx * ny * nz;
    size_t off = 0;
    p->o_scalars = off;
    off = align_up(off + sizeof(double) * (pp::SC_COUNT + 4 * (size_t)batch));
    p->o_partial = off;
    off = align_up(off + sizeof(double) * 3 * p->nper * batch);
    for (int i = 0; i < p->ntab; ++i) {
        p->o_tab[i] = off;
        off = align_up(off + p->tb[i].blob.size());
    }
    p->o_S = off;
    off = align_up(off + p->elem * (size_t)batch * p->slots * nz * ny);
    p->o_r = off;   // refined, rows over 512: the double residual
    if (dtype == PP_F32_REFINED && !pp::res_fused_supported(nx)) off = align_up(off + sizeof(double) * n * batch);
    p->o_u0 = off;
    if (dtype == PP_F32_REFINED) off = align_up(off + sizeof(float) * n * batch);
    p->o_lo = off;
    off = align_up(off + sizeof(cplx<double>) * (size_t)batch * p->nlo * nz * ny);
    if (p->zsegs > 0) {
        // segment end values (2 per segment) and couplings (2 per segment),
        // per (batch, slot, entry)
        p->o_seg = off;
        off = align_up(off + p->elem * (size_t)batch * p->slots * ny * p->zsegs * 4);
    }
    if (p->zsplit > 0) {
        for (int i = 0; i < p->ntab; ++i) {
            p->o_zb[i] = off;
            const size_t el = (i == 0) ? p->elem : sizeof(cplx<double>);
            off = align_up(off + el * (size_t)batch * p->slots * 2 * ny);
        }
    }
    p->ws_bytes = off;
    *out = p;
    return PP_OK;
}

pp_status pp_plan_set_gauge(pp_plan p, pp_gauge gauge) {
    if (!p) return PP_ERR_ARG;
    if (gauge != PP_GAUGE_MEAN && gauge != PP_GAUGE_PIN && gauge != PP_GAUGE_PIN_RAW) return PP_ERR_ARG;
    p->gauge = gauge;
    return PP_OK;
}

pp_status pp_plan_set_zsolver(pp_plan p, pp_zsolver solver) {
    if (!p || (solver != PP_ZSOLVER_THOMAS && solver != PP_ZSOLVER_PCR && solver != PP_ZSOLVER_CR)) return PP_ERR_ARG;
    if (solver == PP_ZSOLVER_PCR || solver == PP_ZSOLVER_CR) {
        if (p->bz0 == pp::BC_P) return PP_ERR_BC;
        if (p->nz > 4096 || p->ny > 512) return PP_ERR_SIZE;
    }
    p->zsolver = (int)solver;
    if (p->dtype == PP_F32_REFINED) set_mixed_slots(p);
    return PP_OK;
}

pp_status pp_plan_set_zsplit(pp_plan p, pp_zsplit mode) {
    if (!p || (mode != PP_ZSPLIT_AUTO && mode != PP_ZSPLIT_OFF && mode != PP_ZSPLIT_ON && mode != PP_ZSPLIT_SEG))
        return PP_ERR_ARG;
    if (mode == PP_ZSPLIT_ON && p->zsplit == 0) return (p->bz0 == pp::BC_P) ? PP_ERR_BC : PP_ERR_SIZE;
    if (mode == PP_ZSPLIT_SEG && p->zsegs == 0) return (p->bz0 == pp::BC_P) ? PP_ERR_BC : PP_ERR_SIZE;
    p->zsplit_mode = (int)mode;
    return PP_OK;
}

pp_status pp_plan_set_refinement(pp_plan p, double tol, int max_iter) {
    if (!p || !(tol >= 0.0) || max_iter < 0) return PP_ERR_ARG;
    p->ir_tol = tol;
    p->ir_max = max_iter;
    return PP_OK;
}

size_t pp_plan_workspace_bytes(pp_plan p) { return p ? p->ws_bytes : 0; }

pp_status pp_solve(pp_plan p, const void* f, void* u, void* workspace, void* stream) {
    return dispatch(p, f, u, workspace, stream, false);
}

pp_status pp_solve_adjoint(pp_plan p, const void* g, void* out, void* workspace, void* stream) {
    return dispatch(p, g, out, workspace, stream, true);
}

pp_status pp_solve_bc(pp_plan p, const void* f, const void* const faces[6], void* u, void* workspace,
                      void* stream) {
    return dispatch(p, f, u, workspace, stream, false, faces);
}

pp_status pp_plan_last_info(pp_plan p, int* ir_iters, double* removed_mean, double* final_rel_update) {
    if (!p) return PP_ERR_ARG;
    if (ir_iters) *ir_iters = p->last_iters;
    if (final_rel_update) *final_rel_update = p->last_rel;
    if (!p->last_ws) {
        if (removed_mean)
            for (int b = 0; b < p->batch; ++b) removed_mean[b] = 0.0;
        return PP_OK;
    }
    std::vector<double> sc(pp::SC_COUNT + 4 * (size_t)p->batch);
    if (hipStreamSynchronize(p->last_stream) != hipSuccess) return PP_ERR_HIP;
    if (hipMemcpy(sc.data(), (unsigned char*)p->last_ws + p->o_scalars, sizeof(double) * sc.size(),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return PP_ERR_HIP;
    bool finite = std::isfinite(sc[pp::SC_MAXF]);
    for (int b = 0; b < p->batch; ++b) {
        const double mu = sc[pp::SC_COUNT + 3 * p->batch + b];
        finite = finite && std::isfinite(mu);
        if (removed_mean) removed_mean[b] = p->last_projected ? mu : 0.0;
    }
    return finite ? PP_OK : PP_ERR_NONFINITE;
}

pp_status pp_plan_set_timing(pp_plan p, int on) {
    if (!p) return PP_ERR_ARG;
    p->timing = on != 0;
    return PP_OK;
}

pp_status pp_plan_kernel_times(pp_plan p, double* ms, int* launches, int reset) {
    if (!p) return PP_ERR_ARG;
    const pp_status st = collect(p);
    if (st != PP_OK) return st;
    for (int g = 0; g < 4; ++g) {
        if (ms) ms[g] = p->kms[g];
        if (launches) launches[g] = p->kcount[g];
        if (reset) {
            p->kms[g] = 0.0;
            p->kcount[g] = 0;
        }
    }
    return PP_OK;
}

pp_status pp_solve_noalloc(pp_plan p, const void* f, void* u, void* stream) {
    if (!p || !f || !u) return PP_ERR_ARG;
    if (p->ws_bytes > pp::kScratchBytes) return PP_ERR_SCRATCH;
    void* ws = nullptr;
    if (pp::scratch_buffer(&ws) != hipSuccess) return PP_ERR_HIP;
    // no timing events here: creating them is a runtime allocation
    const bool timing = p->timing;
    p->timing = false;
    const pp_status st = dispatch(p, f, u, ws, stream, false);
    p->timing = timing;
    return st;
}

pp_status pp_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || bytes % 16 != 0 || ((uintptr_t)src % 16) != 0 || ((uintptr_t)dst % 16) != 0)
        return PP_ERR_ARG;
    if (overlap(src, bytes, dst, bytes)) return PP_ERR_ALIAS;
    if (bytes == 0) return PP_OK;
    return pp::launch_stream_copy(src, dst, bytes, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? PP_OK
                                                                                                      : PP_ERR_HIP;
}

void pp_plan_destroy(pp_plan p) {
    if (!p) return;
    (void)collect(p);
    forget_plan(p);
    delete p;
}

const char* pp_status_string(pp_status st) {
    switch (st) {
        case PP_OK: return "ok";
        case PP_ERR_ARG: return "invalid argument";
        case PP_ERR_BC: return "unsupported boundary conditions";
        case PP_ERR_SIZE: return "unsupported grid size";
        case PP_ERR_ALIAS: return "arrays overlap";
        case PP_ERR_WORKSPACE: return "workspace null or misaligned";
        case PP_ERR_HIP: return "HIP runtime error";
        case PP_ERR_NOT_CONVERGED: return "refinement did not converge";
        case PP_ERR_NONFINITE: return "non-finite value in the source";
        case PP_ERR_SCRATCH: return "problem needs more workspace than the fixed no-alloc buffer holds";
    }
    return "unknown status";
}

}  // extern "C"
