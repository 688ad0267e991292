// regpass.hip -- register-resident separable passes of the K-type products
// (Alg 2; the consistent mass and the other operator sets with their own
// coefficient rows), u^h (Alg 3), the load f^r (Alg 4) and the gradient force
// (Alg B.1) on cubic 3D boxes of 32, 48, 64, 80, 96, 128 and 256 points per
// axis: FP32 with the linear basis at every one of them and the quadratic
// basis at 64 and 128, FP64 with the linear basis at 32, 48, 64, 128 and 256.
//
// A complex line packs two adjacent real lines of one field: the real part is
// line w, the imaginary part line w+1.  Every 1D kernel array t_e is real
// (Eq 77-78), so one complex convolution convolves both lines at once and no
// spectral separation is needed; t_e is even or odd in its offset, so its
// spectrum is real or imaginary and one float per frequency describes it.
//
// A complex line of L points is owned by a group of lanes that hold it in
// registers; the layouts of 64 and 128 points are:
//   G8<R>: 8 lanes, lane t holds points t + 8m (m < R, L = 8R).  A transform
//          is a DFT-R in registers, a twiddle, one transpose through LDS and
//          DFT-8s in registers (four-step FFT).
//   G16:   16 lanes, lane t holds points t + 16m (m < 8, L = 128): a DFT-8,
//          a twiddle, one transpose through LDS, a radix-2 step between the
//          two lane halves by a DPP row rotation, a twiddle and a DFT-8.
//          Twice the waves of G8<16> at half the registers, so more latency
//          is hidden; a setup-time measurement picks between the two.
// Either way the data crosses LDS once per transform instead of once per
// radix stage, and the spectral products, the inverse transforms and the
// pointwise stage of the middle pass all act on registers.  The other lengths
// use the P x Q layouts (GPQ) and, at 256 points, also a 32-lane layout with
// two transposes (G32); they run only with the line-constant middle pass.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

#include "fcrkpm_impl.hpp"

namespace fcrkpm {
namespace {

typedef cplx<float> cf;

constexpr int kRT = 256;             // threads per workgroup

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a * e^{-DIR 2 pi i j / 16}, j a compile-time constant after unrolling
template <int DIR, typename T>
__device__ __forceinline__ cplx<T> mul_w16(cplx<T> a, int j)
{
    T c, s;
    if constexpr (sizeof(T) == 4) {
        constexpr float C[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                 0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                                 -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                                 0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
        c = C[j & 15];
        s = C[(j + 12) & 15];  // sin(x) = cos(x - pi/2)
    } else {
        constexpr double C[16] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                                  0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
                                  -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
                                  0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
        c = C[j & 15];
        s = C[(j + 12) & 15];
    }
    const T ds = DIR > 0 ? s : -s;
    return cplx<T>{a.x * c + a.y * ds, a.y * c - a.x * ds};
}

// in-place DFT-16 in natural order, as 4 x 4 with internal twiddles
template <int DIR, typename T>
__device__ __forceinline__ void dft16(cplx<T>* v)
{
    cplx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
        dft4<T, DIR>(a[n2]);
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1)
            if (n2 > 0) a[n2][k1] = mul_w16<DIR>(a[n2][k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4<T, DIR>(b);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dftR_reg(cplx<T>* v)
{
    if constexpr (R == 16) dft16<DIR>(v);
    else dft8<T, DIR>(v);
}

template <int DIR, typename T>
__device__ __forceinline__ cplx<T> twid(const cplx<T>* tw, int j)
{
    const cplx<T> w = tw[j];
    return DIR > 0 ? w : cplx<T>{w.x, -w.y};
}

// Forward transform of the group's line.  In: v[m] = x[t + 8m].  Out:
// v[8j + k2] = X[t + 8j + R k2] (j < R/8, k2 < 8).
template <int R, typename T>
__device__ __forceinline__ void g8_fwd(cplx<T> (&v)[R], int t, cplx<T>* xb, const cplx<T>* tw)
{
    constexpr int KPL = R / 8;
    dftR_reg<R, +1>(v);
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) v[k1] = cmul(v[k1], twid<+1>(tw, t * k1));
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) xb[k1 * 9 + t] = v[k1];
    wave_sync();
#pragma unroll
    for (int j = 0; j < KPL; ++j)
#pragma unroll
        for (int n = 0; n < 8; ++n) v[8 * j + n] = xb[(t + 8 * j) * 9 + n];
    wave_sync();
#pragma unroll
    for (int j = 0; j < KPL; ++j) dft8<T, +1>(v + 8 * j);
}

// Unnormalised inverse: the layout of fwd's output in, x[t + 8m] in v[m] out.
template <int R, typename T>
__device__ __forceinline__ void g8_inv(cplx<T> (&v)[R], int t, cplx<T>* xb, const cplx<T>* tw)
{
    constexpr int KPL = R / 8;
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
        dft8<T, -1>(v + 8 * j);
#pragma unroll
        for (int n1 = 1; n1 < 8; ++n1) v[8 * j + n1] = cmul(v[8 * j + n1], twid<-1>(tw, n1 * (t + 8 * j)));
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) xb[(t + 8 * j) * 9 + n1] = v[8 * j + n1];
    }
    wave_sync();
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) v[k1] = xb[k1 * 9 + t];
    wave_sync();
    dftR_reg<R, -1>(v);
}

// the value of lane t ^ 8 within the lane's row of 16 (DPP row rotation by 8;
// every lane has a source, so no old value is needed)
__device__ __forceinline__ float swap8(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x128, 0xF, 0xF, true));
}
__device__ __forceinline__ double swap8(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0x128, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x128, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The twiddles one G16 lane needs, fixed for the whole kernel: the forward
// W_128^{t k1} (k1 = 1..7), the W_16^{tl h} of its half (1 on h = 0) and the
// inverse W_128^{-(tl + 8h) (t & 7)} (tl = 0..7).  Computed once per lane from
// the LDS table, so the transforms read no twiddles and select nothing.
template <typename T = float>
struct G16Tw {
    typedef cplx<T> cf;
    cf f_[7], h_[7], i_[8];
    __device__ __forceinline__ void make(int t, const cf* tw)
    {
        const int k1 = t & 7, hh = t >> 3;
#pragma unroll
        for (int j = 1; j < 8; ++j) {
            f_[j - 1] = tw[t * j];
            const cf w = mul_w16<+1>(cf{T(1), T(0)}, j);
            h_[j - 1] = hh ? w : cf{T(1), T(0)};
        }
#pragma unroll
        for (int tl = 0; tl < 8; ++tl) i_[tl] = twid<-1>(tw, (tl + 8 * hh) * k1);
    }
    __device__ __forceinline__ cf f(int j) const { return f_[j - 1]; }
    __device__ __forceinline__ cf h(int j) const { return h_[j - 1]; }
    __device__ __forceinline__ cf i(int tl) const { return i_[tl]; }
};

// The same twiddles read from the LDS table when needed (fewer registers, for
// kernels that hold many fields)
template <typename T = float>
struct G16TwL {
    typedef cplx<T> cf;
    const cf* tw;
    int t;
    __device__ __forceinline__ void make(int lane, const cf* table)
    {
        tw = table;
        t = lane;
    }
    __device__ __forceinline__ cf f(int j) const { return tw[t * j]; }
    __device__ __forceinline__ cf h(int j) const
    {
        const cf w = mul_w16<+1>(cf{T(1), T(0)}, j);
        return (t >> 3) ? w : cf{T(1), T(0)};
    }
    __device__ __forceinline__ cf i(int tl) const { return twid<-1>(tw, (tl + 8 * (t >> 3)) * (t & 7)); }
};

// G16 forward transform (L = 128).  In: v[m] = x[t + 16m].  Out: v[i] =
// X[t + 16i].  With t = k1 + 8h the steps are a DFT-8 over m, the twiddle
// W_128^{t k1}, a transpose giving lane (k1, h) the values of lanes
// 8h .. 8h+7 at k1, a radix-2 step across h, the twiddle W_16^{tl h} and a
// DFT-8 over the lane offset tl.
template <class TW, typename T>
__device__ __forceinline__ void g16_fwd(cplx<T> (&v)[8], int t, cplx<T>* xb, const TW& w)
{
    typedef cplx<T> cf;
    dft8<T, +1>(v);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) v[k1] = cmul(v[k1], w.f(k1));
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) xb[k1 * 17 + t] = v[k1];
    wave_sync();
    const int k1 = t & 7, h = t >> 3;
#pragma unroll
    for (int tl = 0; tl < 8; ++tl) v[tl] = xb[k1 * 17 + 8 * h + tl];
    wave_sync();
    const T s = h ? T(-1) : T(1);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const cf u = {swap8(v[i].x), swap8(v[i].y)};
        v[i] = cf{u.x + s * v[i].x, u.y + s * v[i].y};
    }
#pragma unroll
    for (int tl = 1; tl < 8; ++tl) v[tl] = cmul(v[tl], w.h(tl));
    dft8<T, +1>(v);
}

// G16 unnormalised inverse: v[i] = X[t + 16i] in, v[m] = x[t + 16m] out (the
// steps of g16_fwd reversed, with conjugate twiddles).
template <class TW, typename T>
__device__ __forceinline__ void g16_inv(cplx<T> (&v)[8], int t, cplx<T>* xb, const TW& w)
{
    typedef cplx<T> cf;
    const int k1 = t & 7, h = t >> 3;
    dft8<T, -1>(v);
#pragma unroll
    for (int tl = 1; tl < 8; ++tl) v[tl] = cmulc(v[tl], w.h(tl));
    const T s = h ? T(-1) : T(1);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const cf u = {swap8(v[i].x), swap8(v[i].y)};
        v[i] = cf{u.x + s * v[i].x, u.y + s * v[i].y};
    }
#pragma unroll
    for (int tl = 0; tl < 8; ++tl) xb[k1 * 17 + tl + 8 * h] = cmul(v[tl], w.i(tl));
    wave_sync();
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = xb[j * 17 + t];
    wave_sync();
    dft8<T, -1>(v);
}

// The lane's values of the axis's kernel spectra T_e (e < NE), each divided
// by L (the 1/L of the inverse transform): T_e is real for even e and
// imaginary for odd e (t_e is even or odd), so one float per frequency
// describes it.  G16 holds its 8 frequencies of each in registers; G8 reads
// them from the LDS copy.
template <int NE, typename T = float>
struct SpecRegs {
    T s[NE][8];
    template <class Lay>
    __device__ __forceinline__ void fetch(const T* tab, int t)
    {
#pragma unroll
        for (int e = 0; e < NE; ++e)
#pragma unroll
            for (int i = 0; i < 8; ++i) s[e][i] = tab[e * Lay::L + Lay::freq(t, i)];
    }
    template <class Lay>
    __device__ __forceinline__ void bind(const T*, int) {}
    template <class Lay, int E>
    __device__ __forceinline__ T e(int i) const { return s[E][i]; }
};
template <typename T = float>
struct SpecLds {
    const T* trl;
    int t;
    template <class Lay>
    __device__ __forceinline__ void fetch(const T*, int) {}
    template <class Lay>
    __device__ __forceinline__ void bind(const T* tab, int lane)
    {
        trl = tab;
        t = lane;
    }
    template <class Lay, int E>
    __device__ __forceinline__ T e(int i) const { return trl[E * Lay::L + Lay::freq(t, i)]; }
};

// Line layouts: lanes per complex line, points per lane, the spatial row of
// point m and the frequency of spectral slot i held by lane t, the LDS
// complex values of one group's transpose buffer (the group stride is 8 mod
// 32 so the groups of a wave spread over the banks), and the geometry of the
// staging buffer of strided passes (TP, SS, STAGE; see stage_move).
// G8 reads its twiddles from the LDS table as it goes
template <typename T = float>
struct LdsTw {
    const cplx<T>* tw;
    __device__ __forceinline__ void make(int, const cplx<T>* table) { tw = table; }
};

template <int R>
struct G8 {
    static constexpr int LANES = 8, PTS = R, SPTS = R, L = 8 * R, XS = R == 16 ? 168 : 72;
    static constexpr int GROUPS = kRT / LANES, LINES = 2 * GROUPS;
    static constexpr int TP = GROUPS + 1, SS = LANES * TP, STAGE = PTS * SS;
    template <typename T = float>
    using TwT = LdsTw<T>;
    typedef TwT<float> Tw;
    template <int NE, typename T = float>
    using Spec = SpecLds<T>;
    static __device__ __forceinline__ int row(int t, int m) { return t + 8 * m; }
    static __device__ __forceinline__ int freq(int t, int i) { return t + 8 * (i / 8) + R * (i % 8); }
    static __device__ __forceinline__ int lane_of(int k) { return k % 8; }
    static __device__ __forceinline__ int slot_of(int k)
    {
        constexpr int Q = R / 8;
        const int rem = k / 8;
        return 8 * (rem % Q) + rem / Q;
    }
    template <typename T>
    static __device__ __forceinline__ void fwd(cplx<T> (&v)[R], int t, cplx<T>* xb, const LdsTw<T>& w) { g8_fwd<R>(v, t, xb, w.tw); }
    template <typename T>
    static __device__ __forceinline__ void inv(cplx<T> (&v)[R], int t, cplx<T>* xb, const LdsTw<T>& w) { g8_inv<R>(v, t, xb, w.tw); }
};
struct G16 {
    static constexpr int LANES = 16, PTS = 8, SPTS = 8, L = 128, XS = 136;
    static constexpr int GROUPS = kRT / LANES, LINES = 2 * GROUPS;
    static constexpr int TP = GROUPS + 1, SS = LANES * TP, STAGE = PTS * SS;
    template <typename T = float>
    using TwT = G16Tw<T>;
    typedef TwT<float> Tw;
    template <int NE, typename T = float>
    using Spec = SpecRegs<NE, T>;
    static __device__ __forceinline__ int row(int t, int m) { return t + 16 * m; }
    static __device__ __forceinline__ int freq(int t, int i) { return t + 16 * i; }
    static __device__ __forceinline__ int lane_of(int k) { return k % 16; }
    static __device__ __forceinline__ int slot_of(int k) { return k / 16; }
    template <typename T, class TW>
    static __device__ __forceinline__ void fwd(cplx<T> (&v)[8], int t, cplx<T>* xb, const TW& w) { g16_fwd(v, t, xb, w); }
    template <typename T, class TW>
    static __device__ __forceinline__ void inv(cplx<T> (&v)[8], int t, cplx<T>* xb, const TW& w) { g16_inv(v, t, xb, w); }
};
// G16 geometry with twiddles and spectra read from LDS (for the kernel that
// holds the most fields)
struct G16L {
    static constexpr int LANES = 16, PTS = 8, SPTS = 8, L = 128, XS = 136;
    static constexpr int GROUPS = kRT / LANES, LINES = 2 * GROUPS;
    static constexpr int TP = GROUPS + 1, SS = LANES * TP, STAGE = PTS * SS;
    template <typename T = float>
    using TwT = G16TwL<T>;
    typedef TwT<float> Tw;
    template <int NE, typename T = float>
    using Spec = SpecLds<T>;
    static __device__ __forceinline__ int row(int t, int m) { return t + 16 * m; }
    static __device__ __forceinline__ int freq(int t, int i) { return t + 16 * i; }
    static __device__ __forceinline__ int lane_of(int k) { return k % 16; }
    static __device__ __forceinline__ int slot_of(int k) { return k / 16; }
    template <typename T, class TW>
    static __device__ __forceinline__ void fwd(cplx<T> (&v)[8], int t, cplx<T>* xb, const TW& w) { g16_fwd(v, t, xb, w); }
    template <typename T, class TW>
    static __device__ __forceinline__ void inv(cplx<T> (&v)[8], int t, cplx<T>* xb, const TW& w) { g16_inv(v, t, xb, w); }
};

// In-register DFT of P points in natural order, DIR = +1 forward.  Prime
// sizes and 4, 8, 16 have their own butterflies; P = A B (6, 10, 12) takes
// the DFT-A of the B interleaved subsequences, the twiddles W_P^(n2 k1)
// (from the L-point table of the axis, P dividing L) and the DFT-Bs.
template <int P, int DIR, typename T>
__device__ __forceinline__ void dft_small(cplx<T>* v, const cplx<T>* twL, int L)
{
    if constexpr (P == 1) {
        return;
    } else if constexpr (P == 16) {
        dft16<DIR>(v);
    } else if constexpr (P == 2 || P == 3 || P == 4 || P == 5 || P == 7 || P == 8) {
        dftR<T, DIR, P>(v);
    } else {
        constexpr int A = (P % 4 == 0) ? 4 : 2, B = P / A;
        static_assert(A * B == P && (B == 3 || B == 5), "DFT size without a decomposition");
        cplx<T> y[A][B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) {
            cplx<T> a[A];
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) a[n1] = v[B * n1 + n2];
            dftR<T, DIR, A>(a);
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1)
                y[k1][n2] = (n2 * k1 == 0) ? a[k1] : cmul(a[k1], twid<DIR>(twL, n2 * k1 * (L / P)));
        }
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            cplx<T> b[B];
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) b[n2] = y[k1][n2];
            dftR<T, DIR, B>(b);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = b[k2];
        }
    }
}

// Line layout for L = P Q: Q lanes per complex line, lane t holding points
// t + Q m (m < P).  Forward: a DFT-P over m in registers, the twiddle
// W_L^(t k1), one transpose through LDS that hands lane t the Q values of
// each k1 = t + Q j < P (j < J = ceil(P / Q)), and a DFT-Q per such k1: slot
// j Q + k2 then holds X[k1 + P k2].  Slots with k1 >= P hold nothing during
// the spectral stage (their results are never read); when P < Q some lanes
// idle through the DFT-Q stage.  The inverse runs the steps backwards with
// conjugate twiddles.  G8<8> is the square case P = Q = 8.
template <int P_, int Q_>
struct GPQ {
    static constexpr int P = P_, Q = Q_;
    static constexpr int LANES = Q, L = P * Q, J = (P + Q - 1) / Q;
    static constexpr int SPTS = P, PTS = (P > J * Q) ? P : J * Q;
    static constexpr int XP = Q + 1;  // transpose pitch (conflict-free rows)
    static constexpr int XS = (P * XP > PTS * LANES) ? P * XP : PTS * LANES;
    static constexpr int GROUPS = kRT / LANES, LINES = 2 * GROUPS;
    static constexpr int TP = GROUPS + 1, SS = LANES * TP, STAGE = SPTS * SS;
    template <typename T = float>
    using TwT = LdsTw<T>;
    typedef TwT<float> Tw;
    template <int NE, typename T = float>
    using Spec = SpecLds<T>;
    static __device__ __forceinline__ int row(int t, int m) { return t + Q * m; }
    static __device__ __forceinline__ int freq(int t, int i)
    {
        const int k1 = t + Q * (i / Q);
        return k1 < P ? k1 + P * (i % Q) : 0;
    }
    static __device__ __forceinline__ int lane_of(int k) { return (k % P) % Q; }
    static __device__ __forceinline__ int slot_of(int k) { return ((k % P) / Q) * Q + k / P; }
    template <typename T>
    static __device__ __forceinline__ void dftq(cplx<T>* v)
    {
        if constexpr (Q == 16) dft16<+1>(v);
        else dft8<T, +1>(v);
    }
    template <typename T>
    static __device__ __forceinline__ void idftq(cplx<T>* v)
    {
        if constexpr (Q == 16) dft16<-1>(v);
        else dft8<T, -1>(v);
    }
    template <typename T>
    static __device__ __forceinline__ void fwd(cplx<T> (&v)[PTS], int t, cplx<T>* xb, const LdsTw<T>& w)
    {
        dft_small<P, +1>(v, w.tw, L);
#pragma unroll
        for (int k1 = 1; k1 < P; ++k1) v[k1] = cmul(v[k1], twid<+1>(w.tw, t * k1));
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) xb[k1 * XP + t] = v[k1];
        wave_sync();
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int k1 = t + Q * j;
            if (k1 < P) {
#pragma unroll
                for (int n2 = 0; n2 < Q; ++n2) v[j * Q + n2] = xb[k1 * XP + n2];
            }
        }
        wave_sync();
#pragma unroll
        for (int j = 0; j < J; ++j) dftq(v + j * Q);
    }
    template <typename T>
    static __device__ __forceinline__ void inv(cplx<T> (&v)[PTS], int t, cplx<T>* xb, const LdsTw<T>& w)
    {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            idftq(v + j * Q);
            const int k1 = t + Q * j;
            if (k1 < P) {
#pragma unroll
                for (int n2 = 0; n2 < Q; ++n2)
                    xb[k1 * XP + n2] = n2 == 0 ? v[j * Q] : cmul(v[j * Q + n2], twid<-1>(w.tw, n2 * k1));
            }
        }
        wave_sync();
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) v[k1] = xb[k1 * XP + t];
        wave_sync();
        dft_small<P, -1>(v, w.tw, L);
    }
};

// Line layout for L = 16 P (P = 5, 6: 80 and 96 points) with 16 lanes per
// complex line, the 16-lane layout's transform with a DFT-P first: lane t
// holds points t + 16m (m < P); a DFT-P over m, the twiddle W_L^(t k1), a
// transpose through LDS that gives lane k1 + 8h (k1 < P) the values of lanes
// 8h .. 8h+7 at k1, a radix-2 step between the lane halves (DPP row
// rotation), the twiddle W_16^(tl h) and a DFT-8: lane k1 + 8h then holds
// frequencies k1 + P (h + 2i).  Lanes with k1 >= P idle through the second
// stage.  A lane holds 8 values per field where the 6 x 16 and 5 x 16 P x Q
// layouts hold 16, so FP64 lines fit; tiles are positioned pair by pair as
// the P x Q layouts' are (32 lines do not divide 80 or 96).
template <int P_>
struct G16P {
    static constexpr int P = P_, LANES = 16, PTS = 8, SPTS = P, L = 16 * P, XS = 136;
    static constexpr int GROUPS = kRT / LANES, LINES = 2 * GROUPS;
    static constexpr int TP = GROUPS + 1, SS = LANES * TP, STAGE = SPTS * SS;
    template <typename T = float>
    using TwT = LdsTw<T>;
    typedef TwT<float> Tw;
    template <int NE, typename T = float>
    using Spec = SpecLds<T>;
    static __device__ __forceinline__ int row(int t, int m) { return t + 16 * m; }
    static __device__ __forceinline__ int freq(int t, int i)
    {
        const int k1 = t & 7;
        return k1 < P ? k1 + P * ((t >> 3) + 2 * i) : 0;
    }
    static __device__ __forceinline__ int lane_of(int k) { return k % P + 8 * ((k / P) & 1); }
    static __device__ __forceinline__ int slot_of(int k) { return (k / P) >> 1; }
    template <typename T>
    static __device__ __forceinline__ void fwd(cplx<T> (&v)[8], int t, cplx<T>* xb, const LdsTw<T>& w)
    {
        typedef cplx<T> cf;
        dft_small<P, +1>(v, w.tw, L);
#pragma unroll
        for (int k1 = 1; k1 < P; ++k1) v[k1] = cmul(v[k1], twid<+1>(w.tw, t * k1));
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) xb[k1 * 17 + t] = v[k1];
        wave_sync();
        const int k1 = t & 7, h = t >> 3;
#pragma unroll
        for (int tl = 0; tl < 8; ++tl) v[tl] = xb[k1 * 17 + 8 * h + tl];
        wave_sync();
        const T s = h ? T(-1) : T(1);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const cf u = {swap8(v[i].x), swap8(v[i].y)};
            v[i] = cf{u.x + s * v[i].x, u.y + s * v[i].y};
        }
        if (h) {
#pragma unroll
            for (int tl = 1; tl < 8; ++tl) v[tl] = mul_w16<+1>(v[tl], tl);
        }
        dft8<T, +1>(v);
    }
    template <typename T>
    static __device__ __forceinline__ void inv(cplx<T> (&v)[8], int t, cplx<T>* xb, const LdsTw<T>& w)
    {
        typedef cplx<T> cf;
        const int k1 = t & 7, h = t >> 3;
        dft8<T, -1>(v);
        if (h) {
#pragma unroll
            for (int tl = 1; tl < 8; ++tl) v[tl] = mul_w16<-1>(v[tl], tl);
        }
        const T s = h ? T(-1) : T(1);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const cf u = {swap8(v[i].x), swap8(v[i].y)};
            v[i] = cf{u.x + s * v[i].x, u.y + s * v[i].y};
        }
        // lanes with k1 >= P carry nothing; their rows are never read
        const int kk = k1 < P ? k1 : 0;
#pragma unroll
        for (int tl = 0; tl < 8; ++tl) xb[k1 * 17 + tl + 8 * h] = cmul(v[tl], twid<-1>(w.tw, (tl + 8 * h) * kk));
        wave_sync();
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = xb[j * 17 + t];
        wave_sync();
        dft_small<P, -1>(v, w.tw, L);
    }
};

// Line layout for L = 256 with 32 lanes per complex line: lane t holds points
// t + 32m (m < 8) and, after the forward transform, frequencies t + 32i.
// With t = t1 + 8 t2 (t1 < 8, t2 < 4) and k = k1 + 8 ka + 32 kb (k1 < 8,
// ka < 4, kb < 8) the kernel W_256^(n k) of n = t + 32m factors into
// W_8^(m k1) W_256^(t k1) W_4^(t2 ka) W_32^(t1 ka) W_8^(t1 kb).  Forward: a
// DFT-8 over m in registers, the twiddle W_256^(t k1), a transpose through
// LDS after which lane t1 + 8c holds the four t2 values of k1 = 2c and
// 2c + 1, two DFT-4s over t2, the twiddle W_32^(t1 ka), a second transpose
// after which lane k1 + 8 ka holds the eight t1 values, and a DFT-8 over t1.
// The inverse runs the steps backwards with conjugate twiddles.  A lane keeps
// 8 values per field throughout (the 16 x 16 layout keeps 16), so the
// kernels that hold three or more fields fit twice the waves per SIMD.
struct G32 {
    static constexpr int LANES = 32, PTS = 8, SPTS = 8, L = 256;
    static constexpr int S1 = 36, S2 = 33;  // pitches of the two transposes
    static constexpr int XS = 8 * S1;       // covers both and PTS * LANES
    static constexpr int GROUPS = kRT / LANES, LINES = 2 * GROUPS;
    static constexpr int TP = GROUPS + 1, SS = LANES * TP, STAGE = SPTS * SS;
    template <typename T = float>
    using TwT = LdsTw<T>;
    typedef TwT<float> Tw;
    template <int NE, typename T = float>
    using Spec = SpecLds<T>;
    static __device__ __forceinline__ int row(int t, int m) { return t + 32 * m; }
    static __device__ __forceinline__ int freq(int t, int i) { return t + 32 * i; }
    static __device__ __forceinline__ int lane_of(int k) { return k % 32; }
    static __device__ __forceinline__ int slot_of(int k) { return k / 32; }
    template <typename T>
    static __device__ __forceinline__ void fwd(cplx<T> (&v)[8], int t, cplx<T>* xb, const LdsTw<T>& w)
    {
        dft8<T, +1>(v);
#pragma unroll
        for (int k1 = 1; k1 < 8; ++k1) v[k1] = cmul(v[k1], twid<+1>(w.tw, t * k1));
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) xb[k1 * S1 + t] = v[k1];
        wave_sync();
        const int t1 = t & 7, c = t >> 3;
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int t2 = 0; t2 < 4; ++t2) v[4 * e + t2] = xb[(2 * c + e) * S1 + t1 + 8 * t2];
        wave_sync();
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            dft4<T, +1>(v + 4 * e);
#pragma unroll
            for (int ka = 1; ka < 4; ++ka) v[4 * e + ka] = cmul(v[4 * e + ka], twid<+1>(w.tw, 8 * t1 * ka));
#pragma unroll
            for (int ka = 0; ka < 4; ++ka) xb[t1 * S2 + 2 * c + e + 8 * ka] = v[4 * e + ka];
        }
        wave_sync();
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = xb[j * S2 + t];
        wave_sync();
        dft8<T, +1>(v);
    }
    template <typename T>
    static __device__ __forceinline__ void inv(cplx<T> (&v)[8], int t, cplx<T>* xb, const LdsTw<T>& w)
    {
        dft8<T, -1>(v);
#pragma unroll
        for (int j = 0; j < 8; ++j) xb[j * S2 + t] = v[j];
        wave_sync();
        const int t1 = t & 7, c = t >> 3;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
#pragma unroll
            for (int ka = 0; ka < 4; ++ka) v[4 * e + ka] = xb[t1 * S2 + 2 * c + e + 8 * ka];
        }
        wave_sync();
#pragma unroll
        for (int e = 0; e < 2; ++e) {
#pragma unroll
            for (int ka = 1; ka < 4; ++ka) v[4 * e + ka] = cmul(v[4 * e + ka], twid<-1>(w.tw, 8 * t1 * ka));
            dft4<T, -1>(v + 4 * e);
#pragma unroll
            for (int t2 = 0; t2 < 4; ++t2) xb[(2 * c + e) * S1 + t1 + 8 * t2] = v[4 * e + t2];
        }
        wave_sync();
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) v[k1] = xb[k1 * S1 + t];
        wave_sync();
#pragma unroll
        for (int k1 = 1; k1 < 8; ++k1) v[k1] = cmul(v[k1], twid<-1>(w.tw, t * k1));
        dft8<T, -1>(v);
    }
};

template <class Lay>
struct is_gpq : std::false_type {};
template <int P, int Q>
struct is_gpq<GPQ<P, Q>> : std::true_type {};
template <int P>
struct is_gpq<G16P<P>> : std::true_type {};
// layouts that run only with the line-constant middle pass
template <class Lay>
struct lineconst_only : std::integral_constant<bool, is_gpq<Lay>::value || std::is_same<Lay, G32>::value> {};

// Term structure of the K d passes (Eq 55, 77-78): each term convolves input
// `in` of a pass with the kernel t_e (part 1) or the reflected t_e (part 2)
// and adds the result to output `out`.  One table per basis (3D, monomials in
// graded order); reg_path_ok checks the pass programs of the basis against
// the table before the register path is used.
struct RTerm {
    int out, in, e;
};
struct RPass {
    int nin, nout, nterm;
    RTerm t[10];
};
// linear basis: 1, x, y, z
struct Lin3 {
    static constexpr int S = 4, NE = 2, DEGREE = 1;
    static constexpr RPass p1[3] = {
        {1, 2, 2, {{0, 0, 0}, {1, 0, 1}}},
        {2, 3, 3, {{0, 0, 0}, {1, 1, 0}, {2, 0, 1}}},
        {3, 4, 4, {{0, 0, 0}, {1, 1, 0}, {2, 2, 0}, {3, 0, 1}}}};
    static constexpr RPass p2[3] = {
        {2, 1, 2, {{0, 0, 0}, {0, 1, 1}}},
        {3, 2, 3, {{0, 0, 0}, {0, 2, 1}, {1, 1, 0}}},
        {4, 3, 4, {{0, 0, 0}, {0, 3, 1}, {1, 1, 0}, {2, 2, 0}}}};
};
// quadratic basis: 1, x, y, z, x^2, xy, xz, y^2, yz, z^2
struct Quad3 {
    static constexpr int S = 10, NE = 3, DEGREE = 2;
    static constexpr RPass p1[3] = {
        {1, 3, 3, {{0, 0, 0}, {1, 0, 1}, {2, 0, 2}}},
        {3, 6, 6, {{0, 0, 0}, {1, 1, 0}, {2, 0, 1}, {3, 2, 0}, {4, 1, 1}, {5, 0, 2}}},
        {6, 10, 10, {{0, 0, 0}, {1, 1, 0}, {2, 2, 0}, {3, 0, 1}, {4, 3, 0}, {5, 4, 0}, {6, 1, 1},
                     {7, 5, 0}, {8, 2, 1}, {9, 0, 2}}}};
    static constexpr RPass p2[3] = {
        {3, 1, 3, {{0, 0, 0}, {0, 1, 1}, {0, 2, 2}}},
        {6, 3, 6, {{0, 0, 0}, {0, 2, 1}, {0, 5, 2}, {1, 1, 0}, {1, 4, 1}, {2, 3, 0}}},
        {10, 6, 10, {{0, 0, 0}, {0, 3, 1}, {0, 9, 2}, {1, 1, 0}, {1, 6, 1}, {2, 2, 0}, {2, 8, 1},
                     {3, 4, 0}, {4, 5, 0}, {5, 7, 0}}}};
};

template <class B, int PART, int J>
constexpr const RPass& rpass() { return PART == 1 ? B::p1[J] : B::p2[J]; }

// index of the N-th term of output O in the pass (-1 past the last)
template <class B, int PART, int J, int O, int N>
constexpr int term_of()
{
    const RPass& P = rpass<B, PART, J>();
    int n = 0;
    for (int k = 0; k < P.nterm; ++k)
        if (P.t[k].out == O) {
            if (n == N) return k;
            ++n;
        }
    return -1;
}

// Y (+)= the spectrum of term K applied to its input: T_e Z for part 1, the
// reflected kernel's spectrum (T_e for even e, its conjugate for odd e) for
// part 2.  T_e is real for even e and imaginary for odd e (one float each).
template <class Lay, class B, int PART, int J, int K, bool FIRST, int NIN, int R, class Sp, typename T>
__device__ __forceinline__ void apply_term(const cplx<T> (&Z)[NIN][R], cplx<T> (&Y)[R], const Sp& sp)
{
    typedef cplx<T> cf;
    constexpr RTerm tm = rpass<B, PART, J>().t[K];
    static_assert(tm.in >= 0 && tm.in < NIN, "term input");
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const T a = sp.template e<Lay, tm.e>(i);
        const cf z = Z[tm.in][i];
        cf v;
        if constexpr ((tm.e & 1) == 0) v = cf{a * z.x, a * z.y};
        else if constexpr (PART == 1) v = cf{-a * z.y, a * z.x};
        else v = cf{a * z.y, -a * z.x};
        if constexpr (FIRST) Y[i] = v;
        else Y[i] = cf{Y[i].x + v.x, Y[i].y + v.y};
    }
}

template <class Lay, class B, int PART, int J, int O, int NIN, int R, class Sp, typename T, int... N>
__device__ __forceinline__ void combine_o(const cplx<T> (&Z)[NIN][R], cplx<T> (&Y)[R], const Sp& sp,
                                          std::integer_sequence<int, N...>)
{
    static_assert(term_of<B, PART, J, O, 0>() >= 0, "every output has a term");
    ((term_of<B, PART, J, O, N>() >= 0
          ? apply_term<Lay, B, PART, J, (term_of<B, PART, J, O, N>() >= 0 ? term_of<B, PART, J, O, N>() : 0),
                       N == 0>(Z, Y, sp)
          : void()),
     ...);
}

template <class Lay, class B, int PART, int J, int NIN, int R, class Sp, typename T, int... O>
__device__ __forceinline__ void combine_sel(const cplx<T> (&Z)[NIN][R], int o, cplx<T> (&Y)[R], const Sp& sp,
                                            std::integer_sequence<int, O...>)
{
    ((o == O ? combine_o<Lay, B, PART, J, O>(Z, Y, sp, std::make_integer_sequence<int, 3>{}) : void()),
     ...);
}

// Spectra of output o of pass (PART, J) from the input spectra Z (fwd's
// layout).  o is constant once the caller's loop over the outputs is
// unrolled, so the selection folds away.
template <class Lay, class B, int PART, int J, int NIN, int R, class Sp, typename T>
__device__ __forceinline__ void combine(const cplx<T> (&Z)[NIN][R], int o, cplx<T> (&Y)[R], const Sp& sp)
{
    combine_sel<Lay, B, PART, J>(Z, o, Y, sp, std::make_integer_sequence<int, rpass<B, PART, J>().nout>{});
}

template <typename T>
struct RArgsT {
    const T* in;              // real fields fstride apart (or the field masked by mask_in)
    const uint8_t* mask_in;
    T* out;
    const uint8_t* mask_out;  // masked single-field store (and dot), else NULL
    long fstride;             // floats between fields
    long in_rb, out_rb;       // floats between right-hand sides (blockIdx.y)
    long st;                  // element stride of the axis; 1 for x
    const T* tr;              // [3][L]: Re T_0 / L, Im T_1 / L, Re T_2 / L of the axis
    const cplx<T>* tw;        // [L] e^{-2 pi i j / L}
    double* dot_part;         // masked store: per-workgroup partial of out . dot_with
    const T* dot_with;
    long dot_stride;          // dot_part slots between right-hand sides
    const uint2* nbits;       // middle pass, per lane: .x bit 2m+c set if node c of element
                              // m is interior, .y bit m set if element m reads a record
    const uint32_t* noff;     // middle pass: per lane, its first record
    const float4* rec;        // middle pass: records of kRec floats
    float ci[kMaxNodeConst + 1];  // middle pass, interior nodes: M (linear basis, sym_index
                                  // order) or b^a (a-major) and V (quadratic basis)
    // first x pass inside CG (PUPD): the pending direction update p = r + beta p
    // with beta = (sum of rr_part) / scal[parity], written back to `in`
    const T* rvec;
    const double* rr_part;
    int nrr;
    double* scal;
    int parity;
    const int* act;
};
typedef RArgsT<float> RArgs;

// The pointwise stage of the middle pass (Eq 90-91) regrouped: with B the
// 3 x 4 matrix b^a_q of a node, E_p = V sum_a b^a_p sum_q b^a_q D_q equals
// sum_q M_pq D_q for the symmetric M = V B^T B, whose 10 distinct entries are
// kept in the order (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3).
// Interior nodes share one M; nodes outside the domain have M = 0 (b = 0
// there); every other element has a record with the M of its two nodes
// interleaved -- M_0(n0), M_0(n1), M_1(n0), ... -- 5 float4 per record.
constexpr int kRec = 20;

// position of M_pq (p <= q) in that order
__host__ __device__ constexpr int sym_index(int p, int q)
{
    return 4 * p - p * (p - 1) / 2 + (q - p);
}

// e = M d for the symmetric M of one node
template <typename T>
__device__ __forceinline__ void sym4_apply(const T* M, T d0, T d1, T d2, T d3, T (&e)[4])
{
    e[0] = M[0] * d0 + M[1] * d1 + M[2] * d2 + M[3] * d3;
    e[1] = M[1] * d0 + M[4] * d1 + M[5] * d2 + M[6] * d3;
    e[2] = M[2] * d0 + M[5] * d1 + M[7] * d2 + M[8] * d3;
    e[3] = M[3] * d0 + M[6] * d1 + M[8] * d2 + M[9] * d3;
}

// Position of the workgroup's Lay::LINES real lines: for a strided axis the
// float index of line l0 at point 0 (the lines are adjacent in memory), for
// x the index of line l0's first point.
// A P x Q layout's tile may hold more lines than one row of a strided axis
// (LINES > st on the y axis of 32- or 48-point boxes, or not dividing it), so
// its strided tiles are positioned line by line: the base is the tile's first
// line and each pair of lines (never split by a row end, the box lengths
// being even) finds its own row.
template <class Lay, bool CONTIG>
__device__ __forceinline__ long tile_base(long tile, long st)
{
    const long l0 = tile * Lay::LINES;
    if (CONTIG) return l0 * Lay::L;
    if constexpr (is_gpq<Lay>::value) return l0;
    const long lo = l0 % st, hi = l0 / st;
    return lo + hi * st * Lay::L;
}

// complex element m of group g: lines (2g, 2g+1) of the tile at point row(t, m)
template <class Lay, bool CONTIG>
__device__ __forceinline__ long elem_index(long base, int g, int t, int m, long st)
{
    const int i = Lay::row(t, m);
    if (CONTIG) return base + (long)(2 * g) * Lay::L + i;
    if constexpr (is_gpq<Lay>::value) {
        const uint32_t l = (uint32_t)(base + 2 * g), s = (uint32_t)st;
        return (long)(l % s) + (long)(l / s) * st * Lay::L + (long)i * st;
    }
    return base + 2 * g + (long)i * st;
}

template <typename T>
using vec2_of = typename std::conditional<sizeof(T) == 4, float2, double2>::type;

template <int L, bool CONTIG, typename T>
__device__ __forceinline__ cplx<T> load_pair(const T* p, long idx)
{
    if (CONTIG) return cplx<T>{p[idx], p[idx + L]};
    const vec2_of<T> v = *reinterpret_cast<const vec2_of<T>*>(p + idx);
    return cplx<T>{v.x, v.y};
}

template <int L, bool CONTIG, typename T>
__device__ __forceinline__ void store_pair(T* p, long idx, cplx<T> v)
{
    if (CONTIG) {
        p[idx] = v.x;
        p[idx + L] = v.y;
    } else {
        *reinterpret_cast<vec2_of<T>*>(p + idx) = vec2_of<T>{v.x, v.y};
    }
}

__device__ __forceinline__ double block_sum(double v, double* sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < kRT / 64; ++i) r += sh[i];
    return r;
}

__device__ __forceinline__ long xcd_tile(long b, long nblocks)
{
    if (nblocks % 8 != 0) return b;
    return (b & 7) * (nblocks >> 3) + (b >> 3);
}

// The twiddle table of the axis and, for layouts that read the spectra from
// LDS, the NE spectra: each thread loads its share into registers (fetch)
// and writes it to LDS later (put), so these loads and those of the input
// lines are in flight together.
template <class Lay, int NE, typename T = float>
struct Tables {
    static constexpr int L = Lay::L;
    static constexpr bool SPEC = std::is_same<typename Lay::template Spec<NE, T>, SpecLds<T>>::value;
    static constexpr int NT = (L + kRT - 1) / kRT;                     // twiddles per thread
    static constexpr int NS = SPEC ? (NE * L + kRT - 1) / kRT : 0;     // spectrum values per thread
    static constexpr int LDS_SPEC = SPEC ? NE * L : 1;                 // values of the LDS copy
    cplx<T> w[NT];
    T s[NS > 0 ? NS : 1];
    template <class A>
    __device__ __forceinline__ void fetch(const A& a)
    {
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            const int e = threadIdx.x + i * kRT;
            if (e < L) w[i] = a.tw[e];
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int e = threadIdx.x + i * kRT;
            if (e < NE * L) s[i] = a.tr[e];
        }
    }
    __device__ __forceinline__ void put(cplx<T>* tw, T* trl) const
    {
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            const int e = threadIdx.x + i * kRT;
            if (e < L) tw[e] = w[i];
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int e = threadIdx.x + i * kRT;
            if (e < NE * L) trl[e] = s[i];
        }
        __syncthreads();
    }
};

// Staging buffers of a layout's strided passes: two, alternated, so one
// barrier per move suffices; one for the 32-lane layout, whose 256-point
// tiles would otherwise hold the LDS to two workgroups per CU.
template <class Lay>
constexpr int stage_bufs() { return std::is_same<Lay, G32>::value ? 1 : 2; }

// Strided passes move global memory in a row-major map: thread (gc, tc) =
// (tid % GROUPS, tid / GROUPS) loads and stores the values of layout lane
// (gc, tc), so GROUPS consecutive threads cover a whole row segment of the
// tile (128 bytes) instead of each wave touching LANES rows with a few
// bytes each.  The values cross LDS once between that thread and the lane
// that transforms them: v holds lane (gw, tw)'s values on entry and lane
// (gr, tr)'s on return.  The TP = GROUPS + 1 pitch keeps both the writes
// (consecutive threads vary g) and the reads (consecutive lanes vary t) free
// of bank conflicts.  Callers alternate two buffers, so the barrier of one
// move also orders the reads of the move before it against the next writes.
template <class Lay, typename T>
__device__ __forceinline__ void stage_move(cplx<T> (&v)[Lay::PTS], cplx<T>* buf, int gw, int tw, int gr, int tr)
{
    // with one buffer, the reads of the move before must finish first
    if constexpr (stage_bufs<Lay>() == 1) __syncthreads();
#pragma unroll
    for (int m = 0; m < Lay::SPTS; ++m) buf[m * Lay::SS + tw * Lay::TP + gw] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < Lay::SPTS; ++m) v[m] = buf[m * Lay::SS + tr * Lay::TP + gr];
}

// One separable pass: NIN real fields -> NOUT real fields along the axis.
// LMASK: the single input is masked by mask_in.  SMASK: the single output is
// masked by mask_out and, if dot_part is set, dotted with dot_with.
// TPW tiles per workgroup: the inputs of all of them are loaded up front, so
// the later tiles' loads overlap the earlier tiles' transforms and stores.
template <class Lay, class B, int TPW, bool CONTIG, bool LMASK, bool SMASK, int PART, int J,
          bool PUPD = false, typename T = float>
__global__ __launch_bounds__(kRT) void k_rpass(RArgsT<T> a)
{
    typedef cplx<T> cf;
    constexpr int L = Lay::L, R = Lay::PTS, SP = Lay::SPTS;  // register slots, points per lane
    // FP32 strided passes stage global memory through LDS (row-major map);
    // FP64 ones read their 16-byte pairs directly in the transform layout
    // (64-byte row segments per wave), which keeps their LDS small
    constexpr bool STG = !CONTIG && sizeof(T) == 4;
    constexpr int NIN = rpass<B, PART, J>().nin, NOUT = rpass<B, PART, J>().nout;
    __shared__ cf tw[L];
    __shared__ T trl[Tables<Lay, B::NE, T>::LDS_SPEC];
    __shared__ cf xbuf[Lay::GROUPS * Lay::XS];
    __shared__ double sh[kRT / 64];
    __shared__ cf stage[STG ? stage_bufs<Lay>() : 1][STG ? Lay::STAGE : 1];
    const int tid = threadIdx.x, g = tid / Lay::LANES, t = tid % Lay::LANES;
    const int gc = STG ? tid % Lay::GROUPS : g, tc = STG ? tid / Lay::GROUPS : t;
    const long rhs = blockIdx.y;
    const T* in = a.in + rhs * a.in_rb;
    T* out = a.out + rhs * a.out_rb;
    const long tile0 = xcd_tile(blockIdx.x, gridDim.x) * TPW;
    cf* xb = xbuf + g * Lay::XS;
    // the partials of the pending update's r.r are loaded first (all
    // kRedBlocks slots, without branches): loads complete in order, so the
    // reduction then waits for them alone
    constexpr int NPART = PUPD ? kRedBlocks / kRT : 1;
    double part[NPART];
    if constexpr (PUPD) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) part[k] = a.rr_part[rhs * kRedBlocks + tid + k * kRT];
    }
    Tables<Lay, B::NE, T> tabs;
    tabs.fetch(a);
    typename Lay::template Spec<B::NE, T> sp;
    sp.template fetch<Lay>(a.tr, t);

    cf Z[TPW][NIN][R];
    uint8_t mk[LMASK ? TPW : 1][LMASK ? R : 1][2];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
        for (int f = 0; f < NIN; ++f)
#pragma unroll
            for (int m = 0; m < SP; ++m) {
                const long idx = elem_index<Lay, CONTIG>(base, gc, tc, m, a.st);
                Z[tt][f][m] = load_pair<L, CONTIG>(in + f * a.fstride, idx);
                if constexpr (LMASK) {
                    mk[tt][m][0] = a.mask_in[idx];
                    mk[tt][m][1] = a.mask_in[idx + (CONTIG ? L : 1)];
                }
            }
    }

    // the pending CG direction update p = r + beta p of the masked input: the
    // same reduction and arithmetic as the stand-alone update kernel, so the
    // iterates are bit for bit the same.  p and r are loaded before the
    // reduction, so their latency overlaps it.
    if constexpr (PUPD) {
        static_assert(LMASK && NIN == 1, "the update applies to the masked single input");
        cf Rv[TPW][R];
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
            const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
            for (int m = 0; m < SP; ++m)
                Rv[tt][m] = load_pair<L, CONTIG>(a.rvec + rhs * a.in_rb,
                                                 elem_index<Lay, CONTIG>(base, gc, tc, m, a.st));
        }
        if (a.act[rhs] != 0) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < NPART; ++k)
                if (tid + k * kRT < a.nrr) v += part[k];
            const double rr_new = block_sum(v, sh);
            const double rr_old = a.scal[rhs * kScal + a.parity];
            const T beta = rr_old > 0.0 ? T(rr_new / rr_old) : T(0);
            if (blockIdx.x == 0 && tid == 0) a.scal[rhs * kScal + 1 - a.parity] = rr_new;
#pragma unroll
            for (int tt = 0; tt < TPW; ++tt) {
                const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
                for (int m = 0; m < SP; ++m) {
                    const cf pv = Z[tt][0][m], rv = Rv[tt][m];
                    Z[tt][0][m] = cf{rv.x + beta * pv.x, rv.y + beta * pv.y};
                    store_pair<L, CONTIG>(const_cast<T*>(in), elem_index<Lay, CONTIG>(base, gc, tc, m, a.st),
                                          Z[tt][0][m]);
                }
            }
        }
    }
    if constexpr (LMASK) {
        static_assert(NIN == 1, "a masked input is a single field");
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
#pragma unroll
            for (int m = 0; m < SP; ++m) {
                const cf v = Z[tt][0][m];
                Z[tt][0][m] = cf{mk[tt][m][0] ? v.x : T(0), mk[tt][m][1] ? v.y : T(0)};
            }
        }
    }
    // the masked store's mask bytes and the dot's other vector, loaded after
    // the fields (loads complete in order) so they arrive during the transforms
    uint8_t mo[SMASK ? TPW : 1][SMASK ? R : 1][2];
    T dwv[SMASK ? TPW : 1][SMASK ? R : 1][2];
    if constexpr (SMASK) {
        const T* dw = a.dot_with + rhs * a.out_rb;
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
            const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
            for (int m = 0; m < SP; ++m) {
                const long idx = elem_index<Lay, CONTIG>(base, gc, tc, m, a.st);
                const long idx1 = idx + (CONTIG ? L : 1);
                mo[tt][m][0] = a.mask_out[idx];
                mo[tt][m][1] = a.mask_out[idx1];
                if (a.dot_part) {
                    dwv[tt][m][0] = dw[idx];
                    dwv[tt][m][1] = dw[idx1];
                }
            }
        }
    }
    tabs.put(tw, trl);
    sp.template bind<Lay>(trl, t);
    typename Lay::template TwT<T> lw;
    lw.make(t, tw);
    double dacc = 0.0;
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
    const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
    for (int f = 0; f < NIN; ++f) {
        if constexpr (STG) stage_move<Lay>(Z[tt][f], stage[(tt * (NIN + NOUT) + f) % stage_bufs<Lay>()], gc, tc, g, t);
        Lay::fwd(Z[tt][f], t, xb, lw);
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        cf Y[R];
        combine<Lay, B, PART, J>(Z[tt], o, Y, sp);
        Lay::inv(Y, t, xb, lw);
        if constexpr (STG) stage_move<Lay>(Y, stage[(tt * (NIN + NOUT) + NIN + o) % stage_bufs<Lay>()], g, t, gc, tc);
#pragma unroll
        for (int m = 0; m < SP; ++m) {
            const long idx = elem_index<Lay, CONTIG>(base, gc, tc, m, a.st);
            if constexpr (SMASK) {
                const T v0 = mo[tt][m][0] ? Y[m].x : T(0);
                const T v1 = mo[tt][m][1] ? Y[m].y : T(0);
                store_pair<L, CONTIG>(out, idx, cf{v0, v1});
                if (a.dot_part)
                    dacc += (double)v0 * (double)dwv[tt][m][0] + (double)v1 * (double)dwv[tt][m][1];
            } else {
                store_pair<L, CONTIG>(out + o * a.fstride, idx, Y[m]);
            }
        }
    }
    }
    if constexpr (SMASK) {
        if (a.dot_part) {
            const double s = block_sum(dacc, sh);
            if (tid == 0) a.dot_part[rhs * a.dot_stride + blockIdx.x] = s;
        }
    }
}

// Middle pass of K d along the last axis (strided), linear basis in 3D
// (s = 4): the part-1 convolutions give D_q, the pointwise stage forms
// E_p = V sum_a b^a_p sum_q b^a_q D_q at every node (Eq 90-91, Alg 2) as
// sum_q M_pq D_q, and the part-2 convolutions of E_p follow -- all in
// registers.
template <class Lay, int TPW, int NIN, int NOUT>
__global__ __launch_bounds__(kRT) void k_rmid(RArgs a)
{
    constexpr int L = Lay::L, R = Lay::PTS;
    constexpr int S = 4;
    __shared__ cf tw[L];
    __shared__ float trl[Tables<Lay, Lin3::NE>::LDS_SPEC];
    __shared__ cf xbuf[Lay::GROUPS * Lay::XS];
    __shared__ cf stage[2][Lay::STAGE];
    const int tid = threadIdx.x, g = tid / Lay::LANES, t = tid % Lay::LANES;
    const int gc = tid % Lay::GROUPS, tc = tid / Lay::GROUPS;
    const long rhs = blockIdx.y;
    const float* in = a.in + rhs * a.in_rb;
    float* out = a.out + rhs * a.out_rb;
    const long tile0 = xcd_tile(blockIdx.x, gridDim.x) * TPW;
    cf* xb = xbuf + g * Lay::XS;
    Tables<Lay, Lin3::NE> tabs;
    tabs.fetch(a);
    typename Lay::template Spec<Lin3::NE> sp;
    sp.template fetch<Lay>(a.tr, t);

    cf Z[TPW][NIN][R];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const long base = tile_base<Lay, false>(tile0 + tt, a.st);
#pragma unroll
        for (int f = 0; f < NIN; ++f)
#pragma unroll
            for (int m = 0; m < R; ++m)
                Z[tt][f][m] = load_pair<L, false>(in + f * a.fstride,
                                                  elem_index<Lay, false>(base, gc, tc, m, a.st));
    }
    // the pointwise stage's node classes, loaded after the fields (loads
    // complete in order, so the first transforms do not wait for them)
    uint2 bw[TPW];
    uint32_t offv[TPW];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const long lane = (tile0 + tt) * kRT + tid;
        bw[tt] = a.nbits[lane];
        offv[tt] = a.noff[lane];
    }
    tabs.put(tw, trl);
    sp.template bind<Lay>(trl, t);
    typename Lay::Tw lw;
    lw.make(t, tw);
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
    const long base = tile_base<Lay, false>(tile0 + tt, a.st);
    cf D[S][R];
    {
#pragma unroll
        for (int f = 0; f < NIN; ++f) {
            stage_move<Lay>(Z[tt][f], stage[(tt * (NIN + NOUT) + f) & 1], gc, tc, g, t);
            Lay::fwd(Z[tt][f], t, xb, lw);
        }
#pragma unroll
        for (int q = 0; q < S; ++q) combine<Lay, Lin3, 1, 2>(Z[tt], q, D[q], sp);
    }
    // the records of the first element pair (the rows at the two ends of the
    // line, where the boundary lies) are requested before the inverse
    // transforms, which hide their latency
    float4 pre[2][kRec / 4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int m = u ? R - 1 : 0;
        if ((bw[tt].y >> m) & 1u) {
            const uint32_t km = __popc(bw[tt].y & ((1u << m) - 1u));
            const float4* src = a.rec + (size_t)(offv[tt] + km) * (kRec / 4);
#pragma unroll
            for (int j = 0; j < kRec / 4; ++j) pre[u][j] = src[j];
        }
    }
#pragma unroll
    for (int q = 0; q < S; ++q) Lay::inv(D[q], t, xb, lw);
    // pointwise stage on both lines of every complex element: E = M D per
    // node.  Only lanes whose element reads a record issue loads, so a wave
    // with none (deep interior, or all outside) skips them.  Elements go in
    // pairs m, R-1-m (the rows nearest the two ends of the line first, where
    // the boundary lies), each pair's records loaded together; the empty asm
    // makes the next pair's record index depend on this pair's results, so
    // the compiler cannot hoist every pair's loads to the top and hold all of
    // them in registers at once.
    uint32_t roff = offv[tt];
#pragma unroll
    for (int h = 0; h < R / 2; ++h) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int m = u ? R - 1 - h : h;
            // interior nodes: the shared M (uniform); outside the domain: 0
            float e0[S], e1[S];
            sym4_apply(a.ci, D[0][m].x, D[1][m].x, D[2][m].x, D[3][m].x, e0);
            sym4_apply(a.ci, D[0][m].y, D[1][m].y, D[2][m].y, D[3][m].y, e1);
            const bool i0 = (bw[tt].x >> (2 * m)) & 1u, i1 = (bw[tt].x >> (2 * m + 1)) & 1u;
#pragma unroll
            for (int p = 0; p < S; ++p) {
                e0[p] = i0 ? e0[p] : 0.0f;
                e1[p] = i1 ? e1[p] : 0.0f;
            }
            if ((bw[tt].y >> m) & 1u) {
                const uint32_t km = __popc(bw[tt].y & ((1u << m) - 1u));
                const float4* src = a.rec + (size_t)(roff + km) * (kRec / 4);
                float M0[10], M1[10];
#pragma unroll
                for (int j = 0; j < kRec / 4; ++j) {
                    const float4 f = h == 0 ? pre[u][j] : src[j];
                    M0[2 * j] = f.x;
                    M1[2 * j] = f.y;
                    M0[2 * j + 1] = f.z;
                    M1[2 * j + 1] = f.w;
                }
                sym4_apply(M0, D[0][m].x, D[1][m].x, D[2][m].x, D[3][m].x, e0);
                sym4_apply(M1, D[0][m].y, D[1][m].y, D[2][m].y, D[3][m].y, e1);
            }
#pragma unroll
            for (int p = 0; p < S; ++p) D[p][m] = cf{e0[p], e1[p]};
        }
        asm volatile("" : "+v"(roff) : "v"(D[0][h].x), "v"(D[0][R - 1 - h].x));
    }
#pragma unroll
    for (int p = 0; p < S; ++p) Lay::fwd(D[p], t, xb, lw);
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        cf Y[R];
        combine<Lay, Lin3, 2, 2>(D, o, Y, sp);
        Lay::inv(Y, t, xb, lw);
        stage_move<Lay>(Y, stage[(tt * (NIN + NOUT) + NIN + o) & 1], g, t, gc, tc);
#pragma unroll
        for (int m = 0; m < R; ++m)
            store_pair<L, false>(out + o * a.fstride, elem_index<Lay, false>(base, gc, tc, m, a.st), Y[m]);
    }
    }
}

// Middle pass for the quadratic basis in 3D (s = 10).  The 10 fields D_q do
// not fit in registers at once, so the pointwise stage streams: as each D_q
// leaves its inverse transform, A^a += b^a_q D_q (Eq 90); then each E_p =
// V sum_a b^a_p A^a is formed, transformed and added to the one output it
// feeds (Eq 91, Alg 2).  The D_q are taken in an order that retires the
// inputs early (an input is dead after its last term).  Interior nodes take
// b^a and V from the kernel argument, nodes outside the domain give zero,
// and the other elements read records of kRec2 floats: b^a_q of the two
// nodes interleaved, q-major then a ([q][a][node], 60 floats), then V of both.
constexpr int kRec2 = 64;
constexpr int kQOrder[10] = {4, 5, 7, 1, 6, 2, 8, 0, 3, 9};

// A^a += b^a_Q d for element m (d: its two nodes).  Interior nodes use the
// kernel argument, nodes outside the domain add nothing, record elements
// read b^a_Q of both nodes from their record.  The uniform products are
// selected after they are formed, so the compiler has no reason to compute
// them ahead for every element.
template <int Q, int R>
__device__ __forceinline__ void quad_acc(const RArgs& a, uint2 bw, uint32_t off, int m, cf d,
                                         cf (&A)[3][R], bool first)
{
    const bool i0 = (bw.x >> (2 * m)) & 1u, i1 = (bw.x >> (2 * m + 1)) & 1u;
    cf add[3];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const float bq = a.ci[al * 10 + Q];
        add[al] = cf{i0 ? bq * d.x : 0.0f, i1 ? bq * d.y : 0.0f};
    }
    if ((bw.y >> m) & 1u) {
        const uint32_t km = __popc(bw.y & ((1u << m) - 1u));
        const float2* r2 = reinterpret_cast<const float2*>(a.rec) + (size_t)(off + km) * (kRec2 / 2);
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            const float2 b = r2[Q * 3 + al];
            add[al] = cf{b.x * d.x, b.y * d.y};
        }
    }
#pragma unroll
    for (int al = 0; al < 3; ++al) A[al][m] = first ? add[al] : cf{A[al][m].x + add[al].x, A[al][m].y + add[al].y};
}

// E_P = V sum_a b^a_P A^a for element m's two nodes; A^a of element m is
// As[(a R + m) kRT] (this lane's values, parked in LDS)
template <int P, int R>
__device__ __forceinline__ cf quad_e(const RArgs& a, uint2 bw, uint32_t off, int m, const cf* As)
{
    const cf A[3][1] = {{As[(0 * R + m) * kRT]}, {As[(1 * R + m) * kRT]}, {As[(2 * R + m) * kRT]}};
    const bool i0 = (bw.x >> (2 * m)) & 1u, i1 = (bw.x >> (2 * m + 1)) & 1u;
    float e0 = a.ci[P] * A[0][0].x, e1 = a.ci[P] * A[0][0].y;
#pragma unroll
    for (int al = 1; al < 3; ++al) {
        e0 += a.ci[al * 10 + P] * A[al][0].x;
        e1 += a.ci[al * 10 + P] * A[al][0].y;
    }
    cf e = cf{i0 ? a.ci[30] * e0 : 0.0f, i1 ? a.ci[30] * e1 : 0.0f};
    if ((bw.y >> m) & 1u) {
        const uint32_t km = __popc(bw.y & ((1u << m) - 1u));
        const float2* r2 = reinterpret_cast<const float2*>(a.rec) + (size_t)(off + km) * (kRec2 / 2);
        float2 b[3];
#pragma unroll
        for (int al = 0; al < 3; ++al) b[al] = r2[P * 3 + al];
        const float2 v = r2[30];
        float f0 = b[0].x * A[0][0].x, f1 = b[0].y * A[0][0].y;
#pragma unroll
        for (int al = 1; al < 3; ++al) {
            f0 += b[al].x * A[al][0].x;
            f1 += b[al].y * A[al][0].y;
        }
        e = cf{v.x * f0, v.y * f1};
    }
    return e;
}

// one part-2 term of the quadratic middle pass: E_p from A, its forward
// transform, and Y (+)= the reflected kernel's spectrum times it
template <class Lay, int O, int N, int TPW_UNUSED = 0>
__device__ __forceinline__ void quad_out_term(const RArgs& a, uint2 bw, uint32_t off, const cf* A,
                                              cf (&Y)[Lay::PTS], int t, cf* xb, const typename Lay::Tw& lw,
                                              const typename Lay::template Spec<Quad3::NE>& sp)
{
    constexpr int K = term_of<Quad3, 2, 2, O, N>();
    if constexpr (K >= 0) {
        constexpr int P = Quad3::p2[2].t[K].in;
        cf E[1][Lay::PTS];
        uint32_t roff = off;
#pragma unroll
        for (int m = 0; m < Lay::PTS; ++m) {
            E[0][m] = quad_e<P, Lay::PTS>(a, bw, roff, m, A);
            // the next element's record index depends on this result, so the
            // compiler cannot hoist every element's loads and hold them all
            if (m & 1) asm volatile("" : "+v"(roff) : "v"(E[0][m].x));
        }
        Lay::fwd(E[0], t, xb, lw);
        // the term reads input 0 of this one-field view
        constexpr RTerm tm = Quad3::p2[2].t[K];
#pragma unroll
        for (int i = 0; i < Lay::PTS; ++i) {
            const float c = sp.template e<Lay, tm.e>(i);
            const cf z = E[0][i];
            cf w;
            if constexpr ((tm.e & 1) == 0) w = cf{c * z.x, c * z.y};
            else w = cf{c * z.y, -c * z.x};
            if constexpr (N == 0) Y[i] = w;
            else Y[i] = cf{Y[i].x + w.x, Y[i].y + w.y};
        }
    }
}

template <class Lay, int TPW>
__global__ __launch_bounds__(kRT) void k_rmid2(RArgs a)
{
    using B = Quad3;
    constexpr int L = Lay::L, R = Lay::PTS;
    constexpr int NIN = B::p1[2].nin, NOUT = B::p2[2].nout;
    static_assert(B::p1[2].nout == B::S && B::p2[2].nin == B::S, "middle pass fields");
    static_assert(TPW == 1, "one tile per workgroup");
    __shared__ cf tw[L];
    __shared__ float trl[Tables<Lay, B::NE>::LDS_SPEC];
    __shared__ cf xbuf[Lay::GROUPS * Lay::XS];
    // every input waits in its own staging slot until its first term, so only
    // the inputs in use occupy registers; the outputs reuse the first two slots
    __shared__ cf slot[NIN][Lay::STAGE];
    const int tid = threadIdx.x, g = tid / Lay::LANES, t = tid % Lay::LANES;
    const int gc = tid % Lay::GROUPS, tc = tid / Lay::GROUPS;
    const long rhs = blockIdx.y;
    const float* in = a.in + rhs * a.in_rb;
    float* out = a.out + rhs * a.out_rb;
    const long tile = xcd_tile(blockIdx.x, gridDim.x);
    const long base = tile_base<Lay, false>(tile, a.st);
    cf* xb = xbuf + g * Lay::XS;
    Tables<Lay, B::NE> tabs;
    tabs.fetch(a);
    typename Lay::template Spec<B::NE> sp;
    sp.template fetch<Lay>(a.tr, t);
    {
        cf raw[NIN][R];
#pragma unroll
        for (int f = 0; f < NIN; ++f)
#pragma unroll
            for (int m = 0; m < R; ++m)
                raw[f][m] = load_pair<L, false>(in + f * a.fstride, elem_index<Lay, false>(base, gc, tc, m, a.st));
#pragma unroll
        for (int f = 0; f < NIN; ++f)
#pragma unroll
            for (int m = 0; m < R; ++m) slot[f][m * Lay::SS + tc * Lay::TP + gc] = raw[f][m];
    }
    const long lane = tile * kRT + tid;
    const uint2 bw = a.nbits[lane];
    const uint32_t off = a.noff[lane];
    tabs.put(tw, trl);  // its barrier also orders the slot writes before the reads
    sp.template bind<Lay>(trl, t);
    typename Lay::Tw lw;
    lw.make(t, tw);

    // input f in the transform layout, forward transformed
    auto take = [&](int f, cf (&Zf)[R]) {
#pragma unroll
        for (int m = 0; m < R; ++m) Zf[m] = slot[f][m * Lay::SS + t * Lay::TP + g];
        Lay::fwd(Zf, t, xb, lw);
    };
    cf Z[NIN][R];
    cf A[3][R];
#pragma unroll
    for (int k = 0; k < B::S; ++k) {
        const int q = kQOrder[k];
        // the first use of an input brings it in from its slot
        if (k == 0) take(3, Z[3]);
        if (k == 1) take(4, Z[4]);
        if (k == 2) take(5, Z[5]);
        if (k == 3) take(1, Z[1]);
        if (k == 5) take(2, Z[2]);
        if (k == 7) take(0, Z[0]);
        cf D[R];
        combine<Lay, B, 1, 2>(Z, q, D, sp);
        Lay::inv(D, t, xb, lw);
        uint32_t roff = off;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            // q is constant after unrolling; quad_acc takes it as a template argument
            switch (q) {
                case 0: quad_acc<0>(a, bw, roff, m, D[m], A, k == 0); break;
                case 1: quad_acc<1>(a, bw, roff, m, D[m], A, k == 0); break;
                case 2: quad_acc<2>(a, bw, roff, m, D[m], A, k == 0); break;
                case 3: quad_acc<3>(a, bw, roff, m, D[m], A, k == 0); break;
                case 4: quad_acc<4>(a, bw, roff, m, D[m], A, k == 0); break;
                case 5: quad_acc<5>(a, bw, roff, m, D[m], A, k == 0); break;
                case 6: quad_acc<6>(a, bw, roff, m, D[m], A, k == 0); break;
                case 7: quad_acc<7>(a, bw, roff, m, D[m], A, k == 0); break;
                case 8: quad_acc<8>(a, bw, roff, m, D[m], A, k == 0); break;
                default: quad_acc<9>(a, bw, roff, m, D[m], A, k == 0); break;
            }
            if (m & 1) asm volatile("" : "+v"(roff) : "v"(A[0][m].x));
        }
        // keep the scheduler from computing later D_q early (each would hold
        // another field of registers)
        __builtin_amdgcn_sched_barrier(0);
    }
    // every input has been read from its slot before the outputs reuse them;
    // A waits in the slots after the first two (this lane's own values, so
    // program order suffices), leaving the registers to the output transforms
    __syncthreads();
    cf* As = &slot[2][0] + tid;
    static_assert(3 * R * kRT <= (NIN - 2) * Lay::STAGE, "A fits the free slots");
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int m = 0; m < R; ++m) As[(al * R + m) * kRT] = A[al][m];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        cf Y[R];
        switch (o) {
#define FC_OUT(OO)                                                          \
    case OO:                                                                \
        quad_out_term<Lay, OO, 0>(a, bw, off, As, Y, t, xb, lw, sp);       \
        quad_out_term<Lay, OO, 1>(a, bw, off, As, Y, t, xb, lw, sp);       \
        quad_out_term<Lay, OO, 2>(a, bw, off, As, Y, t, xb, lw, sp);       \
        break;
            FC_OUT(0) FC_OUT(1) FC_OUT(2) FC_OUT(3) FC_OUT(4) default: FC_OUT(5)
#undef FC_OUT
        }
        Lay::inv(Y, t, xb, lw);
        stage_move<Lay>(Y, slot[o & 1], g, t, gc, tc);
#pragma unroll
        for (int m = 0; m < R; ++m)
            store_pair<L, false>(out + o * a.fstride, elem_index<Lay, false>(base, gc, tc, m, a.st), Y[m]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <class Lay>
long blocks_of(const Ctx& c) { return c.nn / Lay::L / Lay::LINES; }
// ------------------------------------------------ line-constant middle pass
// Along a z line of a cube-like domain the node's support neighbourhood, and
// so its moment matrix, b^a and V, only change within floor(a~) nodes of the
// two ends of the domain's z extent (and outside it, where they vanish).
// Away from those few nodes the pointwise matrix M = V B^T B of the line is a
// constant M_L, and a constant pointwise stage commutes with the z
// convolutions: the part-1 z convolutions, E = M_L D and the part-2 z
// convolutions collapse into one 3 x 3 matrix of spectra applied to the three
// input lines (Eq 90-91 with constant coefficients).  The nodes where M
// differs get the difference directly: D_q there from the kernel taps (a few
// neighbours), dE = (M - M_L) D, spread back with the reflected taps.  So the
// middle pass runs 3 forward and 3 inverse transforms per line pair instead
// of 3 + 4 + 4 + 3, and reads one small record per pair instead of records
// per boundary element.  The two real lines of a complex line pair have the
// same M_L except at the x ends of the domain; there the pair's spectra are
// separated with X(k) and conj X(-k) (the packed lines are real).
constexpr int kSymC = 8;                   // correction nodes per line at most
constexpr int kSymW = 16;                  // their window (corrections +- m) at most
constexpr int kSymRec = 20 + 20 * kSymC + 4;  // floats per pair record
constexpr int kSymFlag = kSymRec - 1;      // record slot of the mismatch flag

// Geometry of the corrections, shared by every line (device copy, staged in LDS)
struct SymTab {
    int nc, nw, m, pad;
    int cz[kSymC];           // correction nodes (z), ascending
    int wz[kSymW];           // window nodes: the correction nodes +- m, ascending
    float tap0[8], tap1[8];  // t_0[o], t_1[o] for o = -m .. m
    signed char widx[256];   // window index of every z (-1: not in the window)
    double dtap0[8], dtap1[8];  // the same taps in FP64
};

template <typename T>
__device__ __forceinline__ T tap0_of(const SymTab& tb, int k)
{
    if constexpr (sizeof(T) == 4) return tb.tap0[k];
    else return tb.dtap0[k];
}
template <typename T>
__device__ __forceinline__ T tap1_of(const SymTab& tb, int k)
{
    if constexpr (sizeof(T) == 4) return tb.tap1[k];
    else return tb.dtap1[k];
}
static_assert(sizeof(SymTab) % 4 == 0, "SymTab is copied in words");

template <typename T>
struct SArgs {
    const T* in;
    T* out;
    long fstride, in_rb, out_rb, st;
    const T* tr;           // [2][L]: Re T_0 / L, Im T_1 / L of the axis
    const cplx<T>* tw;
    const int* pidx;       // per pair: its record
    const T* rec;          // records: M-bar (10), dM' (10), per correction node the 10
                           // entries of dM for both lines interleaved, ..., flag
    const SymTab* tab;
};

// inverse of Lay::freq: the lane and slot that hold frequency k
template <class Lay>
__device__ __forceinline__ int freq_lane(int k) { return Lay::lane_of(k); }
template <class Lay>
__device__ __forceinline__ int freq_slot(int k) { return Lay::slot_of(k); }

// w[i] = conj X(-k) where v[i] = X(k), k = freq(t, i): the spectrum of the
// pair's other orientation, from the lane that holds -k (through LDS)
template <class Lay, typename T>
__device__ __forceinline__ void conj_neg(const cplx<T> (&v)[Lay::PTS], cplx<T> (&w)[Lay::PTS], int t, cplx<T>* xb)
{
    typedef cplx<T> cf;
    constexpr int R = Lay::PTS, L = Lay::L;
#pragma unroll
    for (int i = 0; i < R; ++i) xb[i * Lay::LANES + t] = v[i];
    wave_sync();
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int kn = (L - Lay::freq(t, i)) % L;
        const cf z = xb[freq_slot<Lay>(kn) * Lay::LANES + freq_lane<Lay>(kn)];
        w[i] = cf{z.x, -z.y};
    }
    wave_sync();
}

// Y_j (+)= S_j(M) X at the lane's frequencies: S is the part-1 spectra, the
// constant pointwise matrix M (sym_index order) and the reflected part-2
// spectra of the linear basis's z terms multiplied out.  With T_0 = a (real)
// and T_1 = i b (imaginary), D = (a X0, a X1, a X2, i b X0), E = M D and
// Z = (a E0 - i b E3, a E1, a E2); the products carry one factor 1/L (the
// inverse transform's), the stored spectra one each.
template <class Lay, class Sp, bool ADD, typename T>
__device__ __forceinline__ void sym_apply(const cplx<T> (&X)[3][Lay::PTS], cplx<T> (&Y)[3][Lay::PTS], const T* M,
                                          const Sp& sp)
{
    typedef cplx<T> cf;
#pragma unroll
    for (int i = 0; i < Lay::PTS; ++i) {
        const T a = sp.template e<Lay, 0>(i), b = sp.template e<Lay, 1>(i);
        const T A2 = (T)Lay::L * a * a, AB = (T)Lay::L * a * b, B2 = (T)Lay::L * b * b;
        const T s00 = M[0] * A2 + M[9] * B2;
        const T r01 = M[1] * A2, i01 = -M[6] * AB;   // S_01 = M01 a^2 - i M13 a b
        const T r02 = M[2] * A2, i02 = -M[8] * AB;   // S_02 = M02 a^2 - i M23 a b
        const T s11 = M[4] * A2, s12 = M[5] * A2, s22 = M[7] * A2;
        const cf x0 = X[0][i], x1 = X[1][i], x2 = X[2][i];
        const cf y0 = {s00 * x0.x + r01 * x1.x - i01 * x1.y + r02 * x2.x - i02 * x2.y,
                       s00 * x0.y + r01 * x1.y + i01 * x1.x + r02 * x2.y + i02 * x2.x};
        const cf y1 = {r01 * x0.x + i01 * x0.y + s11 * x1.x + s12 * x2.x,
                       r01 * x0.y - i01 * x0.x + s11 * x1.y + s12 * x2.y};
        const cf y2 = {r02 * x0.x + i02 * x0.y + s12 * x1.x + s22 * x2.x,
                       r02 * x0.y - i02 * x0.x + s12 * x1.y + s22 * x2.y};
        if constexpr (ADD) {
            Y[0][i] = cf{Y[0][i].x + y0.x, Y[0][i].y + y0.y};
            Y[1][i] = cf{Y[1][i].x + y1.x, Y[1][i].y + y1.y};
            Y[2][i] = cf{Y[2][i].x + y2.x, Y[2][i].y + y2.y};
        } else {
            Y[0][i] = y0;
            Y[1][i] = y1;
            Y[2][i] = y2;
        }
    }
}

template <class Lay, typename T = float>
__global__ __launch_bounds__(kRT) void k_smid(SArgs<T> a)
{
    typedef cplx<T> cf;
    constexpr int L = Lay::L, R = Lay::PTS, SP = Lay::SPTS;
    constexpr bool STG = sizeof(T) == 4;  // FP64: direct loads in the transform layout
    constexpr int CW = 3 * kSymW + 4 * kSymC;  // per group: window values (later the
                                               // output corrections), then dE
    __shared__ cf tw[L];
    __shared__ T trl[Tables<Lay, Lin3::NE, T>::LDS_SPEC];
    __shared__ cf xbuf[Lay::GROUPS * Lay::XS];
    __shared__ cf stage[STG ? stage_bufs<Lay>() : 1][STG ? Lay::STAGE : 1];
    __shared__ cf cbuf[Lay::GROUPS * CW];
    __shared__ SymTab tb;
    const int tid = threadIdx.x, g = tid / Lay::LANES, t = tid % Lay::LANES;
    const int gc = STG ? tid % Lay::GROUPS : g, tc = STG ? tid / Lay::GROUPS : t;
    const long rhs = blockIdx.y;
    const T* in = a.in + rhs * a.in_rb;
    T* out = a.out + rhs * a.out_rb;
    const long tile = xcd_tile(blockIdx.x, gridDim.x);
    const long base = tile_base<Lay, false>(tile, a.st);
    cf* xb = xbuf + g * Lay::XS;
    cf* cw = cbuf + g * CW;          // [3][kSymW] window values, then output corrections
    cf* ce = cw + 3 * kSymW;         // [4][kSymC] dE at the correction nodes
    Tables<Lay, Lin3::NE, T> tabs;
    tabs.fetch(a);
    typename Lay::template Spec<Lin3::NE, T> sp;
    sp.template fetch<Lay>(a.tr, t);

    cf X[3][R];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int m = 0; m < SP; ++m)
            X[f][m] = load_pair<L, false>(in + f * a.fstride, elem_index<Lay, false>(base, gc, tc, m, a.st));
    // the pair's record: the constant part for every lane, the correction
    // node's entries for the correction lanes
    const long pair = tile * Lay::GROUPS + g;
    const T* rec = a.rec + (size_t)a.pidx[pair] * kSymRec;
    if (tid < (int)(sizeof(SymTab) / 4))
        reinterpret_cast<int*>(&tb)[tid] = reinterpret_cast<const int*>(a.tab)[tid];
    tabs.put(tw, trl);  // its barrier also publishes tb
    sp.template bind<Lay>(trl, t);
    typename Lay::template TwT<T> lw;
    lw.make(t, tw);
    if constexpr (STG) {
#pragma unroll
        for (int f = 0; f < 3; ++f) stage_move<Lay>(X[f], stage[f % stage_bufs<Lay>()], gc, tc, g, t);
    }
    // window values of the three inputs
#pragma unroll
    for (int m = 0; m < SP; ++m) {
        const int wi = tb.widx[Lay::row(t, m)];
        if (wi >= 0) {
#pragma unroll
            for (int f = 0; f < 3; ++f) cw[f * kSymW + wi] = X[f][m];
        }
    }
    T M[10];
#pragma unroll
    for (int e = 0; e < 10; ++e) M[e] = rec[e];
    const bool mismatch = rec[kSymFlag] != T(0);
    wave_sync();
    // dE = (M - M_L) D at the correction nodes, D from the taps (part 1: D(c) =
    // sum_o t[o] X(c - o)); each line of the pair with its own dM
    for (int ci = t; ci < tb.nc; ci += Lay::LANES) {
        const int cz = tb.cz[ci];
        cf D[4] = {};
        for (int o = -tb.m; o <= tb.m; ++o) {
            const int wi = tb.widx[(cz - o + L) % L];
            const T t0 = tap0_of<T>(tb, o + tb.m), t1 = tap1_of<T>(tb, o + tb.m);
            const cf x0 = cw[wi], x1 = cw[kSymW + wi], x2 = cw[2 * kSymW + wi];
            D[0] = cf{D[0].x + t0 * x0.x, D[0].y + t0 * x0.y};
            D[1] = cf{D[1].x + t0 * x1.x, D[1].y + t0 * x1.y};
            D[2] = cf{D[2].x + t0 * x2.x, D[2].y + t0 * x2.y};
            D[3] = cf{D[3].x + t1 * x0.x, D[3].y + t1 * x0.y};
        }
        const T* dm = rec + 20 + 20 * ci;
        T e0[4], e1[4], MA[10], MB[10];
#pragma unroll
        for (int e = 0; e < 10; ++e) {
            MA[e] = dm[2 * e];
            MB[e] = dm[2 * e + 1];
        }
        sym4_apply(MA, D[0].x, D[1].x, D[2].x, D[3].x, e0);
        sym4_apply(MB, D[0].y, D[1].y, D[2].y, D[3].y, e1);
#pragma unroll
        for (int p = 0; p < 4; ++p) ce[p * kSymC + ci] = cf{e0[p], e1[p]};
    }
    // the three inputs, forward transformed (their wave_syncs also order the
    // dE writes above before the reads below)
#pragma unroll
    for (int f = 0; f < 3; ++f) Lay::fwd(X[f], t, xb, lw);
    cf Y[3][R];
    sym_apply<Lay, decltype(sp), false>(X, Y, M, sp);
    if (mismatch) {
        // lines of different M_L: (M_A + M_B)/2 on X(k) and (M_A - M_B)/2 on conj X(-k)
        T dMp[10];
#pragma unroll
        for (int e = 0; e < 10; ++e) dMp[e] = rec[10 + e];
        cf W[3][R];
#pragma unroll
        for (int f = 0; f < 3; ++f) conj_neg<Lay>(X[f], W[f], t, xb);
        sym_apply<Lay, decltype(sp), true>(W, Y, dMp, sp);
    }
    // output corrections at the window nodes (part 2: dZ(z) = sum_c t[c - z] dE(c)),
    // written over the window values, which are no longer needed
    for (int wi = t; wi < tb.nw; wi += Lay::LANES) {
        const int z = tb.wz[wi];
        cf z0 = {}, z1 = {}, z2 = {};
        for (int ci = 0; ci < tb.nc; ++ci) {
            int d = tb.cz[ci] - z;
            if (d > L / 2) d -= L;
            if (d < -L / 2) d += L;
            if (d < -tb.m || d > tb.m) continue;
            const T t0 = tap0_of<T>(tb, d + tb.m), t1 = tap1_of<T>(tb, d + tb.m);
            const cf e0 = ce[ci], e1 = ce[kSymC + ci], e2 = ce[2 * kSymC + ci], e3 = ce[3 * kSymC + ci];
            z0 = cf{z0.x + t0 * e0.x + t1 * e3.x, z0.y + t0 * e0.y + t1 * e3.y};
            z1 = cf{z1.x + t0 * e1.x, z1.y + t0 * e1.y};
            z2 = cf{z2.x + t0 * e2.x, z2.y + t0 * e2.y};
        }
        cw[wi] = z0;
        cw[kSymW + wi] = z1;
        cw[2 * kSymW + wi] = z2;
    }
#pragma unroll
    for (int o = 0; o < 3; ++o) Lay::inv(Y[o], t, xb, lw);
#pragma unroll
    for (int m = 0; m < SP; ++m) {
        const int wi = tb.widx[Lay::row(t, m)];
        if (wi >= 0) {
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                const cf d = cw[o * kSymW + wi];
                Y[o][m] = cf{Y[o][m].x + d.x, Y[o][m].y + d.y};
            }
        }
    }
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        if constexpr (STG) stage_move<Lay>(Y[o], stage[(3 + o) % stage_bufs<Lay>()], g, t, gc, tc);
#pragma unroll
        for (int m = 0; m < SP; ++m)
            store_pair<L, false>(out + o * a.fstride, elem_index<Lay, false>(base, gc, tc, m, a.st), Y[o][m]);
    }
}

// ------------------------------------------------ gradient nonlinearity, line-constant
// The force of N(g) = (1 + kappa |g|^2) g (Alg B.1), the implicit gradient B d,
// u^h (Alg 3) and the load f^r (Alg 4) on the FP64 register path.  Along a z
// line the pointwise stages of these products have constant coefficients away
// from the correction nodes: the gradient A^a = sum_q b^a_q D_q (Eq 15-16)
// with the line's rows B_L (b^a, or the single row b^0 for u^h), and E_p =
// V sum_a b^a_p N^a with C_L = V_L B_L.  So the middle pass applies B_L to the
// part-1 z spectra, transforms back, corrects A at the correction nodes with
// the taps, applies N node by node, transforms N, applies C_L with the
// reflected part-2 spectra, and corrects the output at the window nodes -- 12
// transforms per line pair for the force.  GRAD stops after A and stores its
// ROWS components (B d, or u^h with the row b^0); LOAD starts from a nodal
// field in place of N (f^r with the row b^0: E_p = V b^0_p r).
enum { KN_FORCE = 0, KN_GRAD = 1, KN_LOAD = 2 };

// record geometry for ROWS coefficient rows of 4 entries
template <int ROWS>
struct KnRec {
    static constexpr int NB = 4 * ROWS;                // entries of B_L, and of C_L
    static constexpr int CORR = 4 * NB;                // per correction node: dB, dC of both lines
    static constexpr int HEAD = 4 * NB;                // B mean, B half difference, C mean, C half
    static constexpr int REC = HEAD + CORR * kSymC + 4;
    static constexpr int FLAG = REC - 1;
    static constexpr int LINE = 2 * NB + 2 * NB * kSymC;  // FP64 line record: B_L, C_L, per node dB, dC
};

template <typename T>
struct KArgs {
    const T* in;
    T* out;
    long fstride, in_rb, out_rb, st;
    const T* tr;           // [2][L]: Re T_0 / L, Im T_1 / L of the axis
    const cplx<T>* tw;
    const int* pidx;       // per pair: its record
    const T* rec;          // records (KnRec): B mean, B half difference, C mean, C half
                           // difference, per correction node the entries of dB and dC for
                           // both lines interleaved, ..., flag
    const SymTab* tab;
    T kappa;
    const uint8_t* mask;   // GRAD: the output's mask (zero outside the domain)
};

// Y_a (+)= G_a(B) x_f for input column F of the gradient operator: A^a(k) =
// (B_a0 a + i B_a3 b) X0 + B_a1 a X1 + B_a2 a X2 (B row-major [a][q])
template <class Lay, class Sp, int F, bool SET, int ROWS, typename T>
__device__ __forceinline__ void kn_grad_col(const cplx<T> (&W)[Lay::PTS], cplx<T> (&Y)[ROWS][Lay::PTS],
                                            const T* Bm, const Sp& sp)
{
    typedef cplx<T> cf;
#pragma unroll
    for (int i = 0; i < Lay::PTS; ++i) {
        const T a = sp.template e<Lay, 0>(i), b = sp.template e<Lay, 1>(i);
        const cf w = W[i];
#pragma unroll
        for (int al = 0; al < ROWS; ++al) {
            cf c;
            if constexpr (F == 0) c = cf{Bm[al * 4 + 0] * a, Bm[al * 4 + 3] * b};
            else c = cf{Bm[al * 4 + F] * a, T(0)};
            Y[al][i] = SET ? cf{c.x * w.x - c.y * w.y, c.x * w.y + c.y * w.x}
                           : cf{Y[al][i].x + c.x * w.x - c.y * w.y, Y[al][i].y + c.x * w.y + c.y * w.x};
        }
    }
}

// Z_f += Q_f(C) n_a for input column a of the divergence operator: Z_0 =
// sum_a (C_a0 a - i C_a3 b) N^a, Z_1 = sum_a C_a1 a N^a, Z_2 = sum_a C_a2 a N^a
// (C row-major [a][p] = V b^a_p)
template <class Lay, class Sp, typename T>
__device__ __forceinline__ void kn_div_col(int al, const cplx<T> (&W)[Lay::PTS], cplx<T> (&Z)[3][Lay::PTS],
                                           const T* Cm, const Sp& sp)
{
    typedef cplx<T> cf;
    const T c0 = Cm[al * 4 + 0], c1 = Cm[al * 4 + 1], c2 = Cm[al * 4 + 2], c3 = Cm[al * 4 + 3];
#pragma unroll
    for (int i = 0; i < Lay::PTS; ++i) {
        const T a = sp.template e<Lay, 0>(i), b = sp.template e<Lay, 1>(i);
        const cf w = W[i];
        const cf q0 = {c0 * a, -c3 * b};
        Z[0][i] = cf{Z[0][i].x + q0.x * w.x - q0.y * w.y, Z[0][i].y + q0.x * w.y + q0.y * w.x};
        Z[1][i] = cf{Z[1][i].x + c1 * a * w.x, Z[1][i].y + c1 * a * w.y};
        Z[2][i] = cf{Z[2][i].x + c2 * a * w.x, Z[2][i].y + c2 * a * w.y};
    }
}

// correction index of node z (or -1)
__device__ __forceinline__ int corr_of(const SymTab& tb, int z)
{
    int ci = -1;
    for (int k = 0; k < tb.nc; ++k)
        if (tb.cz[k] == z) ci = k;
    return ci;
}

template <class Lay, typename T, int MODE, int ROWS>
__global__ __launch_bounds__(kRT) void k_smid_kn(KArgs<T> a)
{
    typedef cplx<T> cf;
    typedef KnRec<ROWS> KR;
    constexpr int L = Lay::L, R = Lay::PTS, SP = Lay::SPTS;
    constexpr bool STG = sizeof(T) == 4;
    constexpr int NB = KR::NB;
    constexpr int CW = 3 * kSymW + 4 * kSymC + 3 * kSymC;  // window values (later output
                                                          // corrections), dE, dA (later N)
    static_assert(MODE != KN_FORCE || ROWS == 3, "the force acts on the gradient");
    __shared__ cf tw[L];
    __shared__ T trl[Tables<Lay, Lin3::NE, T>::LDS_SPEC];
    __shared__ cf xbuf[Lay::GROUPS * Lay::XS];
    __shared__ cf stage[STG ? stage_bufs<Lay>() : 1][STG ? Lay::STAGE : 1];
    __shared__ cf cbuf[Lay::GROUPS * CW];
    __shared__ SymTab tb;
    const int tid = threadIdx.x, g = tid / Lay::LANES, t = tid % Lay::LANES;
    const int gc = STG ? tid % Lay::GROUPS : g, tc = STG ? tid / Lay::GROUPS : t;
    const long rhs = blockIdx.y;
    const T* in = a.in + rhs * a.in_rb;
    T* out = a.out + rhs * a.out_rb;
    const long tile = xcd_tile(blockIdx.x, gridDim.x);
    const long base = tile_base<Lay, false>(tile, a.st);
    cf* xb = xbuf + g * Lay::XS;
    cf* cw = cbuf + g * CW;          // [3][kSymW] window values, then output corrections
    cf* ce = cw + 3 * kSymW;         // [4][kSymC] dE at the correction nodes
    cf* ca = ce + 4 * kSymC;         // [ROWS][kSymC] dA, then N, at the correction nodes
    Tables<Lay, Lin3::NE, T> tabs;
    tabs.fetch(a);
    typename Lay::template Spec<Lin3::NE, T> sp;
    sp.template fetch<Lay>(a.tr, t);

    constexpr int NIN = MODE == KN_LOAD ? 1 : 3;
    cf X[3][R];
#pragma unroll
    for (int f = 0; f < NIN; ++f)
#pragma unroll
        for (int m = 0; m < SP; ++m)
            X[f][m] = load_pair<L, false>(in + f * a.fstride, elem_index<Lay, false>(base, gc, tc, m, a.st));
    const long pair = tile * Lay::GROUPS + g;
    const T* rec = a.rec + (size_t)a.pidx[pair] * KR::REC;
    if (tid < (int)(sizeof(SymTab) / 4))
        reinterpret_cast<int*>(&tb)[tid] = reinterpret_cast<const int*>(a.tab)[tid];
    tabs.put(tw, trl);  // its barrier also publishes tb
    sp.template bind<Lay>(trl, t);
    typename Lay::template TwT<T> lw;
    lw.make(t, tw);
    if constexpr (STG) {
#pragma unroll
        for (int f = 0; f < NIN; ++f) stage_move<Lay>(X[f], stage[f % stage_bufs<Lay>()], gc, tc, g, t);
    }
    const bool mismatch = rec[KR::FLAG] != T(0);
    // the gradient's (or u^h's) values, or the nodal input of the load
    cf Y[ROWS][R];
    if constexpr (MODE == KN_LOAD) {
#pragma unroll
        for (int m = 0; m < SP; ++m) Y[0][m] = X[0][m];
    } else {
#pragma unroll
        for (int m = 0; m < SP; ++m) {
            const int wi = tb.widx[Lay::row(t, m)];
            if (wi >= 0) {
#pragma unroll
                for (int f = 0; f < 3; ++f) cw[f * kSymW + wi] = X[f][m];
            }
        }
        wave_sync();
        // dA = (B - B_L) D at the correction nodes, D from the taps; each line of
        // the pair with its own dB
        for (int ci = t; ci < tb.nc; ci += Lay::LANES) {
            const int cz = tb.cz[ci];
            cf D[4] = {};
            for (int o = -tb.m; o <= tb.m; ++o) {
                const int wi = tb.widx[(cz - o + L) % L];
                const T t0 = tap0_of<T>(tb, o + tb.m), t1 = tap1_of<T>(tb, o + tb.m);
                const cf x0 = cw[wi], x1 = cw[kSymW + wi], x2 = cw[2 * kSymW + wi];
                D[0] = cf{D[0].x + t0 * x0.x, D[0].y + t0 * x0.y};
                D[1] = cf{D[1].x + t0 * x1.x, D[1].y + t0 * x1.y};
                D[2] = cf{D[2].x + t0 * x2.x, D[2].y + t0 * x2.y};
                D[3] = cf{D[3].x + t1 * x0.x, D[3].y + t1 * x0.y};
            }
            const T* dm = rec + KR::HEAD + KR::CORR * ci;
#pragma unroll
            for (int al = 0; al < ROWS; ++al) {
                cf s = {};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = al * 4 + q;
                    s = cf{s.x + dm[2 * e] * D[q].x, s.y + dm[2 * e + 1] * D[q].y};
                }
                ca[al * kSymC + ci] = s;
            }
        }
        // the constant part in the spectral domain
#pragma unroll
        for (int f = 0; f < 3; ++f) Lay::fwd(X[f], t, xb, lw);
        {
            T Bm[NB];
#pragma unroll
            for (int e = 0; e < NB; ++e) Bm[e] = rec[e];
            kn_grad_col<Lay, decltype(sp), 0, true, ROWS>(X[0], Y, Bm, sp);
            kn_grad_col<Lay, decltype(sp), 1, false, ROWS>(X[1], Y, Bm, sp);
            kn_grad_col<Lay, decltype(sp), 2, false, ROWS>(X[2], Y, Bm, sp);
        }
        if (mismatch) {
            // lines of different B_L: the half difference on conj X(-k)
            T Bd[NB];
#pragma unroll
            for (int e = 0; e < NB; ++e) Bd[e] = rec[NB + e];
            cf W[R];
            conj_neg<Lay>(X[0], W, t, xb);
            kn_grad_col<Lay, decltype(sp), 0, false, ROWS>(W, Y, Bd, sp);
            conj_neg<Lay>(X[1], W, t, xb);
            kn_grad_col<Lay, decltype(sp), 1, false, ROWS>(W, Y, Bd, sp);
            conj_neg<Lay>(X[2], W, t, xb);
            kn_grad_col<Lay, decltype(sp), 2, false, ROWS>(W, Y, Bd, sp);
        }
#pragma unroll
        for (int al = 0; al < ROWS; ++al) Lay::inv(Y[al], t, xb, lw);
        wave_sync();
        // the values at the correction nodes
#pragma unroll
        for (int m = 0; m < SP; ++m) {
            const int z = Lay::row(t, m);
            if (tb.widx[z] >= 0) {
                const int ci = corr_of(tb, z);
                if (ci >= 0) {
#pragma unroll
                    for (int al = 0; al < ROWS; ++al) {
                        const cf d = ca[al * kSymC + ci];
                        Y[al][m] = cf{Y[al][m].x + d.x, Y[al][m].y + d.y};
                    }
                }
            }
        }
    }
    if constexpr (MODE == KN_GRAD) {
#pragma unroll
        for (int o = 0; o < ROWS; ++o) {
            if constexpr (STG) stage_move<Lay>(Y[o], stage[(NIN + o) % stage_bufs<Lay>()], g, t, gc, tc);
#pragma unroll
            for (int m = 0; m < SP; ++m) {
                // the pair's lines are adjacent: elements idx and idx + 1
                const long idx = elem_index<Lay, false>(base, gc, tc, m, a.st);
                const cf v = Y[o][m];
                store_pair<L, false>(out + o * a.fstride, idx,
                                     cf{a.mask[idx] ? v.x : T(0), a.mask[idx + 1] ? v.y : T(0)});
            }
        }
        return;
    } else {
        // N(A) node by node (each real line on its own), or the nodal input;
        // its values at the correction nodes kept for their dE
        wave_sync();  // the dA reads above before the writes below
#pragma unroll
        for (int m = 0; m < SP; ++m) {
            if constexpr (MODE == KN_FORCE) {
                const T sx = T(1) + a.kappa * (Y[0][m].x * Y[0][m].x + Y[1][m].x * Y[1][m].x +
                                               Y[2][m].x * Y[2][m].x);
                const T sy = T(1) + a.kappa * (Y[0][m].y * Y[0][m].y + Y[1][m].y * Y[1][m].y +
                                               Y[2][m].y * Y[2][m].y);
#pragma unroll
                for (int al = 0; al < ROWS; ++al) Y[al][m] = cf{sx * Y[al][m].x, sy * Y[al][m].y};
            }
            const int z = Lay::row(t, m);
            if (tb.widx[z] >= 0) {
                const int ci = corr_of(tb, z);
                if (ci >= 0) {
#pragma unroll
                    for (int al = 0; al < ROWS; ++al) ca[al * kSymC + ci] = Y[al][m];
                }
            }
        }
        wave_sync();
        // dE = (C - C_L) N at the correction nodes
        for (int ci = t; ci < tb.nc; ci += Lay::LANES) {
            const T* dm = rec + KR::HEAD + KR::CORR * ci + 2 * NB;
            cf n[ROWS];
#pragma unroll
            for (int al = 0; al < ROWS; ++al) n[al] = ca[al * kSymC + ci];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                cf s = {};
#pragma unroll
                for (int al = 0; al < ROWS; ++al) {
                    const int e = al * 4 + p;
                    s = cf{s.x + dm[2 * e] * n[al].x, s.y + dm[2 * e + 1] * n[al].y};
                }
                ce[p * kSymC + ci] = s;
            }
        }
        // the divergence's constant part in the spectral domain
#pragma unroll
        for (int al = 0; al < ROWS; ++al) Lay::fwd(Y[al], t, xb, lw);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int i = 0; i < R; ++i) X[f][i] = cf{};
        {
            T Cm[NB];
#pragma unroll
            for (int e = 0; e < NB; ++e) Cm[e] = rec[2 * NB + e];
#pragma unroll
            for (int al = 0; al < ROWS; ++al) kn_div_col<Lay>(al, Y[al], X, Cm, sp);
        }
        if (mismatch) {
            T Cd[NB];
#pragma unroll
            for (int e = 0; e < NB; ++e) Cd[e] = rec[3 * NB + e];
            cf W[R];
#pragma unroll
            for (int al = 0; al < ROWS; ++al) {
                conj_neg<Lay>(Y[al], W, t, xb);
                kn_div_col<Lay>(al, W, X, Cd, sp);
            }
        }
        wave_sync();  // the dE writes (and the window reads) before what follows
        // output corrections at the window nodes (part 2: dZ(z) = sum_c t[c - z] dE(c))
        for (int wi = t; wi < tb.nw; wi += Lay::LANES) {
            const int z = tb.wz[wi];
            cf z0 = {}, z1 = {}, z2 = {};
            for (int ci = 0; ci < tb.nc; ++ci) {
                int d = tb.cz[ci] - z;
                if (d > L / 2) d -= L;
                if (d < -L / 2) d += L;
                if (d < -tb.m || d > tb.m) continue;
                const T t0 = tap0_of<T>(tb, d + tb.m), t1 = tap1_of<T>(tb, d + tb.m);
                const cf e0 = ce[ci], e1 = ce[kSymC + ci], e2 = ce[2 * kSymC + ci], e3 = ce[3 * kSymC + ci];
                z0 = cf{z0.x + t0 * e0.x + t1 * e3.x, z0.y + t0 * e0.y + t1 * e3.y};
                z1 = cf{z1.x + t0 * e1.x, z1.y + t0 * e1.y};
                z2 = cf{z2.x + t0 * e2.x, z2.y + t0 * e2.y};
            }
            cw[wi] = z0;
            cw[kSymW + wi] = z1;
            cw[2 * kSymW + wi] = z2;
        }
#pragma unroll
        for (int o = 0; o < 3; ++o) Lay::inv(X[o], t, xb, lw);
#pragma unroll
        for (int m = 0; m < SP; ++m) {
            const int wi = tb.widx[Lay::row(t, m)];
            if (wi >= 0) {
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    const cf d = cw[o * kSymW + wi];
                    X[o][m] = cf{X[o][m].x + d.x, X[o][m].y + d.y};
                }
            }
        }
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            if constexpr (STG) stage_move<Lay>(X[o], stage[(NIN + o) % stage_bufs<Lay>()], g, t, gc, tc);
#pragma unroll
            for (int m = 0; m < SP; ++m)
                store_pair<L, false>(out + o * a.fstride, elem_index<Lay, false>(base, gc, tc, m, a.st), X[o][m]);
        }
    }
}

// Setup of the line-constant middle pass, in FP64.  Line l = x + nx y: M(z)
// at every z, the line's M_L = M(zref), a check that M(z) = M_L off the
// correction nodes (to tol of the product's interior scale), and the line
// record M_L, then dM = M(c) - M_L at each correction node c.
__global__ void k_sym_lines(const double* __restrict__ ba, int krows, const double* __restrict__ vol,
                            long nlines, int nz, long nn, int zref, int nc, const int* __restrict__ czl,
                            double tol, double* __restrict__ lrec, int* __restrict__ bad)
{
    constexpr int S = 4;
    const long l = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (l >= nlines) return;
    auto mat = [&](int z, double (&Mz)[10]) {
        const long node = l + (long)z * nlines;
        const double v = vol[node];
        for (int p = 0; p < S; ++p)
            for (int q = p; q < S; ++q) {
                double acc = 0.0;
                for (int al = 0; al < krows; ++al)
                    acc += ba[(long)(al * S + p) * nn + node] * ba[(long)(al * S + q) * nn + node];
                Mz[sym_index(p, q)] = v * acc;
            }
    };
    double ML[10], Mz[10];
    mat(zref, ML);
    double* o = lrec + l * (10 + 10 * kSymC);
    for (int e = 0; e < 10; ++e) o[e] = ML[e];
    int ci = 0;
    for (int z = 0; z < nz; ++z) {
        const bool corr = ci < nc && czl[ci] == z;
        mat(z, Mz);
        if (corr) {
            for (int e = 0; e < 10; ++e) o[10 + 10 * ci + e] = Mz[e] - ML[e];
            ++ci;
        } else {
            for (int e = 0; e < 10; ++e)
                if (fabs(Mz[e] - ML[e]) > tol) atomicOr(bad, 1);
        }
    }
}

// Pair records (FP32): the mean and half difference of the two lines' M_L,
// the correction entries of both lines interleaved, the mismatch flag.  Pairs
// whose lines both equal the reference pair's (to tol) share record 0, which
// the reference pair writes; every other pair owns record 1 + pair.
__global__ void k_sym_pairs(const double* __restrict__ lrec, long npairs, int nc, long pref, double tol,
                            int* __restrict__ pidx, float* __restrict__ rec, double* __restrict__ rec64,
                            int* __restrict__ own)
{
    const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    constexpr int LR = 10 + 10 * kSymC;
    const double* A = lrec + (2 * p) * LR;
    const double* B = A + LR;
    auto write = [&](float* o, double* o64) {
        bool mism = false;
        for (int e = 0; e < 10; ++e) {
            o64[e] = 0.5 * (A[e] + B[e]);
            const double hd = 0.5 * (A[e] - B[e]);
            o64[10 + e] = hd;
            mism = mism || fabs(hd) > tol;
        }
        for (int ci = 0; ci < kSymC; ++ci)
            for (int e = 0; e < 10; ++e) {
                o64[20 + 20 * ci + 2 * e] = ci < nc ? A[10 + 10 * ci + e] : 0.0;
                o64[20 + 20 * ci + 2 * e + 1] = ci < nc ? B[10 + 10 * ci + e] : 0.0;
            }
        for (int k = 20 + 20 * kSymC; k < kSymRec; ++k) o64[k] = 0.0;
        o64[kSymFlag] = mism ? 1.0 : 0.0;
        for (int k = 0; k < kSymRec; ++k) o[k] = (float)o64[k];
    };
    bool same = pref >= 0;
    if (same) {
        const double* RA = lrec + (2 * pref) * LR;
        for (int k = 0; k < 10 + 10 * nc && same; ++k)
            same = fabs(A[k] - RA[k]) <= tol && fabs(B[k] - RA[LR + k]) <= tol;
    }
    write(rec + (size_t)(1 + p) * kSymRec, rec64 + (size_t)(1 + p) * kSymRec);
    if (p == pref) write(rec, rec64);
    pidx[p] = same ? 0 : (int)(1 + p);
    if (!same) atomicAdd(own, 1);
}

struct SymState {
    const double* ba = nullptr;  // coefficient rows the records were built from
    SymTab* tab = nullptr;       // device
    int* pidx = nullptr;         // device, per pair
    float* rec = nullptr;        // device, 1 + pairs records
    double* rec64 = nullptr;     // the same in FP64
    long own = 0;                // pairs with a record of their own
    SymTab htab{};               // host copy of the table
    int zref = -1;               // the reference node of every line
    double tol = 0.0;            // the records' equality tolerance (M's scale)
    // the gradient nonlinearity's records (B_L, C_L = V_L B_L), built on first use
    int kn = 0;                  // 0 not tried, 1 built, -1 unavailable
    int* knpidx = nullptr;
    double* knrec = nullptr;
    int* b0pidx = nullptr;       // the same for the single row b^0 (u^h, f^r)
    double* b0rec = nullptr;
};

// cubic B-spline of Eq 7 at z = |x| / a
double bspline_d(double z)
{
    z = fabs(z);
    if (z <= 0.5) return 2.0 / 3.0 - 4.0 * z * z + 4.0 * z * z * z;
    if (z < 1.0) return 4.0 / 3.0 - 4.0 * z + 4.0 * z * z - 4.0 / 3.0 * z * z * z;
    return 0.0;
}

template <class Lay, typename T>
void run_smid(const Ctx& c, const T* in, long irb, T* out, long orb, int nrhs, hipStream_t st,
              const RegProf& prof)
{
    const SymState& s = *(const SymState*)c.sym;
    SArgs<T> a{};
    a.in = in;
    a.in_rb = irb;
    a.out = out;
    a.out_rb = orb;
    a.fstride = c.nn;
    a.st = (long)c.n[0] * c.n[1];
    if constexpr (sizeof(T) == 4) {
        a.tr = c.rtab32[2];
        a.tw = c.tw32[2];
        a.rec = s.rec;
    } else {
        a.tr = c.rtab64[2];
        a.tw = c.tw64[2];
        a.rec = s.rec64;
    }
    a.pidx = s.pidx;
    a.tab = s.tab;
    const dim3 grid((unsigned)blocks_of<Lay>(c), (unsigned)nrhs), block(kRT);
    hipEvent_t e0, e1;
    prof.events(2, &e0, &e1);
    if (e0) hipExtLaunchKernelGGL((k_smid<Lay, T>), grid, block, 0, st, e0, e1, 0, a);
    else hipLaunchKernelGGL((k_smid<Lay, T>), grid, block, 0, st, a);
}

// launch of pass k, with the sampler's events recorded by the launch itself
template <typename K, typename A>
void rlaunch(const RegProf& prof, int k, K kern, dim3 grid, dim3 block, hipStream_t st, const A& a)
{
    hipEvent_t e0, e1;
    prof.events(k, &e0, &e1);
    if (e0) hipExtLaunchKernelGGL(kern, grid, block, 0, st, e0, e1, 0, a);
    else hipLaunchKernelGGL(kern, grid, block, 0, st, a);
}

template <class Lay, class B, int TPW>
void run_k(const Ctx& c, const float* in, float* out, const uint8_t* mask, int nrhs,
           double* dot_part, const float* dot_with, hipStream_t st, const RegProf& prof,
           const RegPupd* pu)
{
    const long nn = c.nn;
    const long slot_rb = 2L * c.basis_plan.maxpairs * nn;  // floats between rhs in a workspace slot
    float* S1 = reinterpret_cast<float*>(c.work32);
    float* S2 = S1 + slot_rb * c.cap_work;
    const dim3 grid((unsigned)(blocks_of<Lay>(c) / TPW), (unsigned)nrhs), block(kRT);
    auto args = [&](int axis, const float* i, long irb, float* o, long orb) {
        RArgs a{};
        a.in = i;
        a.in_rb = irb;
        a.out = o;
        a.out_rb = orb;
        a.fstride = nn;
        a.st = axis == 0 ? 1 : (axis == 1 ? (long)c.n[0] : (long)c.n[0] * c.n[1]);
        a.tr = c.rtab32[axis];
        a.tw = c.tw32[axis];
        return a;
    };
    // x: u (masked) -> X, in CG with the pending direction update of u = p
    {
        RArgs a = args(0, in, nn, S1, slot_rb);
        a.mask_in = mask;
        if (pu) {
            a.rvec = pu->r;
            a.rr_part = pu->rr_part;
            a.nrr = pu->nrr;
            a.scal = pu->scal;
            a.parity = pu->parity;
            a.act = pu->act;
            rlaunch(prof, 0, k_rpass<Lay, B, TPW, true, true, false, 1, 0, true>, grid, block, st, a);
        } else {
            rlaunch(prof, 0, k_rpass<Lay, B, TPW, true, true, false, 1, 0>, grid, block, st, a);
        }
    }
    // y: X -> XY
    {
        RArgs a = args(1, S1, slot_rb, S2, slot_rb);
        rlaunch(prof, 1, k_rpass<Lay, B, TPW, false, false, false, 1, 1>, grid, block, st, a);
    }
    // z: XY -> D -> E -> part-2 XY
    {
        RArgs a = args(2, S2, slot_rb, S1, slot_rb);
        a.nbits = c.nbits[c.reg_layout];
        a.noff = c.noff[c.reg_layout];
        a.rec = reinterpret_cast<const float4*>(c.nrec[c.reg_layout]);
        if constexpr (B::DEGREE == 1) {
            constexpr bool SYM_LAYOUT = !std::is_same<Lay, G8<16>>::value;
            if constexpr (lineconst_only<Lay>::value) {
                // the other box lengths run only with the line-constant middle pass
                run_smid<Lay, float>(c, S2, slot_rb, S1, slot_rb, nrhs, st, prof);
            } else if (SYM_LAYOUT && sym_active(c)) {
                if constexpr (SYM_LAYOUT) run_smid<Lay, float>(c, S2, slot_rb, S1, slot_rb, nrhs, st, prof);
            } else {
                for (int k = 0; k < 10; ++k) a.ci[k] = c.reg_mi[k];
                rlaunch(prof, 2, k_rmid<Lay, TPW, 3, 3>, grid, block, st, a);
            }
        } else {
            for (int k = 0; k <= kMaxNodeConst; ++k) a.ci[k] = c.cint32[k];
            // same tile geometry; 16-lane lines read their twiddles and spectra from LDS here
            using MidLay = typename std::conditional<std::is_same<Lay, G16>::value, G16L, Lay>::type;
            rlaunch(prof, 2, k_rmid2<MidLay, TPW>, grid, block, st, a);
        }
    }
    // y: XY -> X
    {
        RArgs a = args(1, S1, slot_rb, S2, slot_rb);
        rlaunch(prof, 3, k_rpass<Lay, B, TPW, false, false, false, 2, 1>, grid, block, st, a);
    }
    // x: X -> f (masked), with the optional dot partials
    {
        RArgs a = args(0, S2, slot_rb, out, nn);
        a.mask_out = mask;
        a.dot_part = dot_part;
        a.dot_with = dot_with;
        a.dot_stride = (long)grid.x <= kRedBlocks ? kRedBlocks : reg_dot_slots(c);
        rlaunch(prof, 4, k_rpass<Lay, B, TPW, true, false, true, 2, 0>, grid, block, st, a);
    }
}

// The FP64 K product on the register path: the same five passes with FP64
// lines (the 16-lane layout reads its twiddles and spectra from LDS), the
// line-constant middle pass, and the optional p.q partials in the last pass.
template <class Lay>
void run_k64(const Ctx& c, const double* in, double* out, const uint8_t* mask, int nrhs,
             double* dot_part, const double* dot_with, hipStream_t st, const RegProf& prof)
{
    const long nn = c.nn;
    const long slot_rb = 2L * c.basis_plan.maxpairs * nn;  // doubles between rhs in a workspace slot
    double* S1 = reinterpret_cast<double*>(c.work64);
    double* S2 = S1 + slot_rb * c.cap_work;
    const dim3 grid((unsigned)blocks_of<Lay>(c), (unsigned)nrhs), block(kRT);
    auto args = [&](int axis, const double* i, long irb, double* o, long orb) {
        RArgsT<double> a{};
        a.in = i;
        a.in_rb = irb;
        a.out = o;
        a.out_rb = orb;
        a.fstride = nn;
        a.st = axis == 0 ? 1 : (axis == 1 ? (long)c.n[0] : (long)c.n[0] * c.n[1]);
        a.tr = c.rtab64[axis];
        a.tw = c.tw64[axis];
        return a;
    };
    {
        RArgsT<double> a = args(0, in, nn, S1, slot_rb);
        a.mask_in = mask;
        rlaunch(prof, 0, k_rpass<Lay, Lin3, 1, true, true, false, 1, 0, false, double>, grid, block, st, a);
    }
    {
        RArgsT<double> a = args(1, S1, slot_rb, S2, slot_rb);
        rlaunch(prof, 1, k_rpass<Lay, Lin3, 1, false, false, false, 1, 1, false, double>, grid, block, st, a);
    }
    run_smid<Lay, double>(c, S2, slot_rb, S1, slot_rb, nrhs, st, prof);
    {
        RArgsT<double> a = args(1, S1, slot_rb, S2, slot_rb);
        rlaunch(prof, 3, k_rpass<Lay, Lin3, 1, false, false, false, 2, 1, false, double>, grid, block, st, a);
    }
    {
        RArgsT<double> a = args(0, S2, slot_rb, out, nn);
        a.mask_out = mask;
        a.dot_part = dot_part;
        a.dot_with = dot_with;
        a.dot_stride = (long)grid.x <= kRedBlocks ? kRedBlocks : reg_dot_slots(c);
        rlaunch(prof, 4, k_rpass<Lay, Lin3, 1, true, false, true, 2, 0, false, double>, grid, block, st, a);
    }
}

// Node classes of every lane of the middle pass, in its own tile geometry
// (cls: 0 outside the domain, 1 interior, 2 other): the interior bits, the
// elements that need a record (unless both nodes are interior or both
// outside) and their count.
template <class Lay>
__global__ void k_rmid_bits(const uint8_t* __restrict__ cls, long st, long nblk,
                            uint2* __restrict__ bits, uint32_t* __restrict__ count,
                            unsigned long long* __restrict__ nload)
{
    const long n = nblk * kRT;
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < n;
         s += (long)gridDim.x * blockDim.x) {
        const long tile = s / kRT;
        const int lane = (int)(s % kRT), g = lane / Lay::LANES, t = lane % Lay::LANES;
        const long base = tile_base<Lay, false>(tile, st);
        uint32_t w = 0, need = 0;
        for (int m = 0; m < Lay::PTS; ++m) {
            const long idx = elem_index<Lay, false>(base, g, t, m, st);
            const uint8_t c0 = cls[idx], c1 = cls[idx + 1];
            if (c0 == 1) w |= 1u << (2 * m);
            if (c1 == 1) w |= 2u << (2 * m);
            if (!(c0 == c1 && c0 != 2)) need |= 1u << m;
        }
        bits[s] = uint2{w, need};
        const int loads = __popc(need);
        count[s] = (uint32_t)loads;
        if (loads) atomicAdd(nload, (unsigned long long)loads);
    }
}

// The records of every lane's record elements, in lane order, with M formed
// in FP64 from the coefficient rows (row-major, [rows][4][nn]: b^a for K) and
// V and rounded once.
template <class Lay>
__global__ void k_rmid_recs(const uint2* __restrict__ bits, const uint32_t* __restrict__ off,
                            const double* __restrict__ ba, const double* __restrict__ vol, long st,
                            long nblk, long nn, int rows, float* __restrict__ rec)
{
    constexpr int S = 4;
    const long n = nblk * kRT;
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < n;
         s += (long)gridDim.x * blockDim.x) {
        const long tile = s / kRT;
        const int lane = (int)(s % kRT), g = lane / Lay::LANES, t = lane % Lay::LANES;
        const long base = tile_base<Lay, false>(tile, st);
        const uint32_t need = bits[s].y;
        long r = off[s];
        for (int m = 0; m < Lay::PTS; ++m) {
            if (!((need >> m) & 1u)) continue;
            const long idx = elem_index<Lay, false>(base, g, t, m, st);
            float* o = rec + r * kRec;
            for (int c = 0; c < 2; ++c) {
                const long node = idx + c;
                const double v = vol[node];
                for (int p = 0; p < S; ++p)
                    for (int q = p; q < S; ++q) {
                        double acc = 0.0;
                        for (int al = 0; al < rows; ++al)
                            acc += ba[(long)(al * S + p) * nn + node] * ba[(long)(al * S + q) * nn + node];
                        o[2 * sym_index(p, q) + c] = (float)(v * acc);
                    }
            }
            ++r;
        }
    }
}

// The records of the quadratic basis: b^a_q of the two nodes, [q][a][node],
// then V of both (kRec2 floats, FP32 copies of the FP64 arrays).
template <class Lay>
__global__ void k_rmid_recs2(const uint2* __restrict__ bits, const uint32_t* __restrict__ off,
                             const double* __restrict__ ba, const double* __restrict__ vol, long st,
                             long nblk, long nn, float* __restrict__ rec)
{
    constexpr int S = 10;
    const long n = nblk * kRT;
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < n;
         s += (long)gridDim.x * blockDim.x) {
        const long tile = s / kRT;
        const int lane = (int)(s % kRT), g = lane / Lay::LANES, t = lane % Lay::LANES;
        const long base = tile_base<Lay, false>(tile, st);
        const uint32_t need = bits[s].y;
        long r = off[s];
        for (int m = 0; m < Lay::PTS; ++m) {
            if (!((need >> m) & 1u)) continue;
            const long idx = elem_index<Lay, false>(base, g, t, m, st);
            float* o = rec + r * kRec2;
            for (int c = 0; c < 2; ++c) {
                const long node = idx + c;
                for (int q = 0; q < S; ++q)
                    for (int al = 0; al < 3; ++al)
                        o[(q * 3 + al) * 2 + c] = (float)ba[(long)(al * S + q) * nn + node];
                o[60 + c] = (float)vol[node];
                o[62 + c] = 0.0f;
            }
            ++r;
        }
    }
}

template <class Lay>
void build_bits(const Ctx& c, const uint8_t* cls, uint2* bits, uint32_t* count,
                unsigned long long* nload, hipStream_t st)
{
    const long str = (long)c.n[0] * c.n[1];
    hipLaunchKernelGGL((k_rmid_bits<Lay>), dim3(256), dim3(256), 0, st, cls, str, blocks_of<Lay>(c),
                       bits, count, nload);
}

template <class Lay>
void build_recs(const Ctx& c, const uint2* bits, const uint32_t* off, float* rec, hipStream_t st)
{
    const long str = (long)c.n[0] * c.n[1];
    if (c.degree == 2)
        hipLaunchKernelGGL((k_rmid_recs2<Lay>), dim3(256), dim3(256), 0, st, bits, off, c.ba_64,
                           c.vol64, str, blocks_of<Lay>(c), c.nn, rec);
    else
        hipLaunchKernelGGL((k_rmid_recs<Lay>), dim3(256), dim3(256), 0, st, bits, off, c.ba_64,
                           c.vol64, str, blocks_of<Lay>(c), c.nn, c.krows, rec);
}

// the pass programs of the basis are exactly the table's terms (in order)
// with coefficient 1/(2L), and -1/(2L) for the odd reflected kernels of part 2
template <class B>
bool plan_matches(const Ctx& c)
{
    if (c.s != B::S) return false;
    const SepPlan& sp = c.basis_plan;
    for (int j = 0; j < 3; ++j) {
        if (c.axes[j] != j) return false;
        const double inv = 1.0 / (2.0 * c.n[j]);
        for (int part = 1; part <= 2; ++part) {
            const SepProg& f = part == 1 ? sp.p1[j] : sp.p2[j];
            const RPass& T = part == 1 ? B::p1[j] : B::p2[j];
            if (f.nin != T.nin || f.nout != T.nout || f.ostart[f.nout] != T.nterm) return false;
            for (int k = 0; k < T.nterm; ++k) {
                const SepTerm& tm = f.t[k];
                const RTerm& want = T.t[k];
                const double coef = (part == 2 && (want.e & 1)) ? -inv : inv;
                if (tm.out != want.out || tm.in != want.in || tm.e != want.e || tm.coef != coef) return false;
                if (k < f.ostart[tm.out] || k >= f.ostart[tm.out + 1]) return false;
            }
        }
    }
    return true;
}

}  // namespace

// box lengths of the P x Q layouts (register path with the line-constant middle pass only)
static bool gpq_length(int L) { return L == 32 || L == 48 || L == 80 || L == 96 || L == 256; }

bool reg_gpq_ok(const Ctx& c)
{
    if (c.dim != 3 || c.naxes != 3 || c.degree != 1) return false;
    const int L = c.n[0];
    if (!gpq_length(L) || c.n[1] != L || c.n[2] != L) return false;
    return plan_matches<Lin3>(c);
}

// layout 0: G8 (8 lanes per line), layout 1: G16 (16 lanes, 128-point lines only);
// for the P x Q lengths, layout 0 has 16 lanes per line (G16P at 80 and 96) and
// layout 1 (80 and 96 only) 8 lanes; 256-point lines: layout 0 is 16 x 16,
// layout 1 the 32-lane G32
int reg_layouts(const Ctx& c)
{
    if (reg_gpq_ok(c)) return (c.n[0] == 80 || c.n[0] == 96 || c.n[0] == 256) ? 2 : 1;
    return c.n[0] == 128 ? 2 : 1;
}

// variant v = layout + 2 (tiles - 1); 8-lane 128-point lines with 2 tiles
// per workgroup need more registers than a wave has, so that one is absent.
// The quadratic basis holds twice the fields: one tile per workgroup, and
// 16 lanes per line at 128 points.
bool reg_variant_ok(const Ctx& c, int v)
{
    if (v < 0 || v > 3 || (v & 1) >= reg_layouts(c)) return false;
    if (reg_gpq_ok(c)) return v < 2;
    if (c.degree == 2) return c.n[0] == 128 ? v == 1 : v == 0;
    return !(c.n[0] == 128 && v == 2);
}

long reg_bits_words(const Ctx& c, int layout)
{
    if (c.n[0] == 128) return (layout ? blocks_of<G16>(c) : blocks_of<G8<16>>(c)) * kRT;
    return blocks_of<G8<8>>(c) * kRT;
}

void launch_reg_bits(const Ctx& c, int layout, const uint8_t* cls, uint2* bits, uint32_t* count,
                     unsigned long long* nload, hipStream_t st)
{
    if (c.n[0] == 128) {
        if (layout) build_bits<G16>(c, cls, bits, count, nload, st);
        else build_bits<G8<16>>(c, cls, bits, count, nload, st);
    } else {
        build_bits<G8<8>>(c, cls, bits, count, nload, st);
    }
}

void launch_reg_recs(const Ctx& c, int layout, const uint2* bits, const uint32_t* off,
                     float* rec, hipStream_t st)
{
    if (c.n[0] == 128) {
        if (layout) build_recs<G16>(c, bits, off, rec, st);
        else build_recs<G8<16>>(c, bits, off, rec, st);
    } else {
        build_recs<G8<8>>(c, bits, off, rec, st);
    }
}

int reg_record_floats(const Ctx& c) { return c.degree == 2 ? kRec2 : kRec; }

bool reg_path_ok(const Ctx& c)
{
    if (c.dim != 3 || c.naxes != 3 || (c.degree != 1 && c.degree != 2)) return false;
    const int L = c.n[0];
    if (L != 64 && L != 128) return false;
    if (c.n[1] != L || c.n[2] != L) return false;
    // the kernels hard-wire the terms of the passes and their coefficients
    return c.degree == 1 ? plan_matches<Lin3>(c) : plan_matches<Quad3>(c);
}

// The layout of a box length: 32 = 4 x 8, 48 = 6 x 8, 80 = G16P<5> or 10 x 8,
// 96 = G16P<6> or 12 x 8, 256 = 16 x 16 or G32.  F(LAY) is called with it.
template <class F>
static void with_gpq(const Ctx& c, F&& f)
{
    switch (c.n[0]) {
        case 32: f(GPQ<4, 8>{}); break;
        case 48: f(GPQ<6, 8>{}); break;
        case 80: if (c.reg_layout) f(GPQ<10, 8>{}); else f(G16P<5>{}); break;
        case 96: if (c.reg_layout) f(GPQ<12, 8>{}); else f(G16P<6>{}); break;
        default: if (c.reg_layout) f(G32{}); else f(GPQ<16, 16>{}); break;
    }
}

// workgroups of one launch (each covers reg_tpw tiles)
int reg_path_blocks(const Ctx& c)
{
    long b;
    if (reg_gpq_ok(c)) {
        with_gpq(c, [&](auto lay) { b = blocks_of<decltype(lay)>(c); });
        return (int)b;
    }
    if (c.n[0] == 128) b = c.reg_layout ? blocks_of<G16>(c) : blocks_of<G8<16>>(c);
    else b = blocks_of<G8<8>>(c);
    return (int)(b / c.reg_tpw);
}

bool sym_ready(const Ctx& c);

long reg_dot_slots(const Ctx& c)
{
    if (c.dim != 3) return kRedBlocks;
    return std::max<long>(kRedBlocks, c.nn / c.n[0] / 16);
}

// FP64 lines fit the registers where a lane holds at most 8 complex values:
// 64^3 and 128^3 boxes, the 32- and 48-point P x Q layouts, the 16-lane
// layouts of 80 and 96 points (G16P) and G32 at 256
bool reg_path64_ok(const Ctx& c)
{
    const bool lay = reg_path_ok(c) || reg_gpq_ok(c);
    return c.degree == 1 && lay && sym_ready(c) && c.rtab64[0] && c.rtab64[1] && c.rtab64[2];
}

long reg_path64_blocks(const Ctx& c)
{
    if (c.n[0] == 32) return blocks_of<GPQ<4, 8>>(c);
    if (c.n[0] == 48) return blocks_of<GPQ<6, 8>>(c);
    if (c.n[0] == 80) return blocks_of<G16P<5>>(c);
    if (c.n[0] == 96) return blocks_of<G16P<6>>(c);
    if (c.n[0] == 256) return blocks_of<G32>(c);
    return c.n[0] == 128 ? blocks_of<G16L>(c) : blocks_of<G8<8>>(c);
}

void launch_reg_k64(const Ctx& c, const double* in, double* out, const uint8_t* mask, int nrhs,
                    double* dot_part, const double* dot_with, hipStream_t st, const RegProf& prof)
{
    if (c.n[0] == 128) run_k64<G16L>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof);
    else if (c.n[0] == 32) run_k64<GPQ<4, 8>>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof);
    else if (c.n[0] == 48) run_k64<GPQ<6, 8>>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof);
    else if (c.n[0] == 80) run_k64<G16P<5>>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof);
    else if (c.n[0] == 96) run_k64<G16P<6>>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof);
    else if (c.n[0] == 256) run_k64<G32>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof);
    else run_k64<G8<8>>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof);
}

void launch_reg_k(const Ctx& c, const float* in, float* out, const uint8_t* mask, int nrhs,
                  double* dot_part, const float* dot_with, hipStream_t st, const RegProf& prof,
                  const RegPupd* pu)
{
#define FC_RUN(LAY)                                                                               \
    do {                                                                                          \
        if (c.reg_tpw == 2) run_k<LAY, Lin3, 2>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu); \
        else run_k<LAY, Lin3, 1>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu);        \
    } while (0)
    if (reg_gpq_ok(c)) {
        with_gpq(c, [&](auto lay) { run_k<decltype(lay), Lin3, 1>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu); });
        return;
    }
    if (c.degree == 2) {
        if (c.n[0] == 128) run_k<G16, Quad3, 1>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu);
        else run_k<G8<8>, Quad3, 1>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu);
    } else if (c.n[0] == 128) {
        if (c.reg_layout) FC_RUN(G16);
        else run_k<G8<16>, Lin3, 1>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu);  // 2 tiles spill
    } else {
        FC_RUN(G8<8>);
    }
#undef FC_RUN
}


// ------------------------------------------------ line-constant middle pass: setup
namespace {
template <typename T>
bool sym_alloc(T*& p, size_t count)
{
    if (hipMalloc((void**)&p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return false;
    }
    return true;
}
template <typename T>
void sym_free(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}
}  // namespace

void sym_release_state(void*& p)
{
    if (!p) return;
    SymState* s = (SymState*)p;
    sym_free(s->tab);
    sym_free(s->pidx);
    sym_free(s->rec);
    sym_free(s->rec64);
    sym_free(s->knpidx);
    sym_free(s->knrec);
    sym_free(s->b0pidx);
    sym_free(s->b0rec);
    delete s;
    p = nullptr;
}

void sym_release(Ctx& c) { sym_release_state(c.sym); }

// the line-constant records exist for the coefficient rows in use (K's, or
// those of an operator set swapped into the context)
bool sym_ready(const Ctx& c)
{
    return c.sym && c.use_sym && ((const SymState*)c.sym)->ba == c.ba_64 && c.degree == 1;
}

// ... and the FP32 product's line layout has the kernel (8-lane 128-point
// lines hold too many values for it)
bool sym_active(const Ctx& c)
{
    return sym_ready(c) && (c.n[0] == 64 || (c.n[0] == 128 && c.reg_layout == 1) || gpq_length(c.n[0]));
}

double sym_pass_bytes(const Ctx& c, int elem_bytes)
{
    const SymState& s = *(const SymState*)c.sym;
    const double pairs = (double)c.nn / c.n[2] / 2.0;
    // three fields in, three out; a record index per pair; the records
    return (double)c.nn * 6.0 * elem_bytes + pairs * 4.0 + (double)(s.own + 1) * kSymRec * elem_bytes;
}

// Builds the line-constant middle pass for K's coefficient rows when every z
// line of the box is constant off the correction nodes (the nodes within
// floor(a~) of the two ends of the domain's z extent, and those outside it);
// leaves c.sym empty otherwise, and the middle pass with records per element
// is used.  Synchronous.
void sym_build(Ctx& c, hipStream_t st)
{
    sym_release(c);
    if (!c.use_sym || c.degree != 1 || c.krows < 1 || !(reg_path_ok(c) || reg_gpq_ok(c)) ||
        c.nconst.bmax < 0.0)
        return;
    const int L = c.n[2], m = c.m[2];
    if (L > 256 || m < 1 || m > 3) return;
    const long nlines = (long)c.n[0] * c.n[1], npairs = nlines / 2;
    // z extent of the domain
    const int ntot = c.n[0] + c.n[1] + c.n[2];
    int* occ = nullptr;
    if (!sym_alloc(occ, ntot)) return;
    std::vector<int> hocc(ntot);
    (void)hipMemsetAsync(occ, 0, sizeof(int) * ntot, st);
    launch_axis_extent(c, c.chi, occ, st);
    (void)hipMemcpyAsync(hocc.data(), occ, sizeof(int) * ntot, hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    sym_free(occ);
    int zlo = -1, zhi = -1;
    for (int z = 0; z < L; ++z)
        if (hocc[c.n[0] + c.n[1] + z]) {
            if (zlo < 0) zlo = z;
            zhi = z;
        }
    if (zlo < 0) return;
    SymTab tab{};
    tab.m = m;
    int zref = -1;
    for (int z = 0; z < L; ++z) {
        if (z < zlo + m || z > zhi - m) {
            if (tab.nc == kSymC) return;
            tab.cz[tab.nc++] = z;
        } else if (zref < 0) {
            zref = z;
        }
    }
    if (zref < 0) return;
    std::vector<char> inw(L, 0);
    for (int i = 0; i < tab.nc; ++i)
        for (int o = -m; o <= m; ++o) inw[(tab.cz[i] + o + L) % L] = 1;
    for (int z = 0; z < 256; ++z) tab.widx[z] = -1;
    for (int z = 0; z < L; ++z)
        if (inw[z]) {
            if (tab.nw == kSymW) return;
            tab.widx[z] = (signed char)tab.nw;
            tab.wz[tab.nw++] = z;
        }
    for (int o = -m; o <= m; ++o) {
        const double w = bspline_d((double)o / c.at[2]);
        tab.tap0[o + m] = (float)w;
        tab.tap1[o + m] = (float)(o * w);
        tab.dtap0[o + m] = w;
        tab.dtap1[o + m] = o * w;
    }
    // the scale of M: the interior nodes' V B^T B
    double mscale = 0.0;
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) {
            double acc = 0.0;
            for (int al = 0; al < c.krows; ++al) acc += c.nconst.b[al * 4 + p] * c.nconst.b[al * 4 + q];
            mscale = std::max(mscale, fabs(c.nconst.v * acc));
        }
    if (!(mscale > 0.0)) return;
    const double tol = 1e-11 * mscale;

    SymState* s = new SymState();
    s->ba = c.ba_64;
    double* lrec = nullptr;
    int* czl = nullptr;
    int* flag = nullptr;
    bool ok = sym_alloc(s->tab, 1) && sym_alloc(s->pidx, npairs) && sym_alloc(s->rec, (size_t)(npairs + 1) * kSymRec) &&
              sym_alloc(s->rec64, (size_t)(npairs + 1) * kSymRec) &&
              sym_alloc(lrec, (size_t)nlines * (10 + 10 * kSymC)) && sym_alloc(czl, kSymC) && sym_alloc(flag, 2);
    if (ok) {
        int hflag[2] = {0, 0};
        (void)hipMemcpyAsync(s->tab, &tab, sizeof(SymTab), hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(czl, tab.cz, sizeof(int) * kSymC, hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(flag, hflag, sizeof(hflag), hipMemcpyHostToDevice, st);
        hipLaunchKernelGGL(k_sym_lines, dim3((unsigned)((nlines + 255) / 256)), dim3(256), 0, st, c.ba_64, c.krows, c.vol64,
                           nlines, L, c.nn, zref, tab.nc, czl, tol, lrec, flag);
        const long pref = ((long)(c.n[0] / 2) + (long)c.n[0] * (c.n[1] / 2)) / 2;
        hipLaunchKernelGGL(k_sym_pairs, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, st, lrec, npairs,
                           tab.nc, pref, tol, s->pidx, s->rec, s->rec64, flag + 1);
        (void)hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, st);
        ok = hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess && hflag[0] == 0;
        s->own = hflag[1];
    }
    (void)hipGetLastError();
    sym_free(lrec);
    sym_free(czl);
    sym_free(flag);
    s->htab = tab;
    s->zref = zref;
    s->tol = tol;
    c.sym = s;
    if (!ok) sym_release(c);
}

// ------------------------------------------------ gradient nonlinearity, u^h, f^r: records and launch
// Line records (FP64) for ROWS coefficient rows: B_L (row-major [a][q]) and
// C_L = V_L B_L, then per correction node B(c) - B_L and C(c) - C_L; any other
// node whose B or C differs from the line's constant (to tol) flags the build
// as unusable.  rows: ROWS x 4 fields nn apart (b^a, or b^0).
template <int ROWS>
__global__ void k_kn_lines(const double* __restrict__ rows, const double* __restrict__ vol, long nlines,
                           int nz, long nn, int zref, int nc, const int* __restrict__ czl,
                           double tolb, double tolc, double* __restrict__ lrec, int* __restrict__ bad)
{
    typedef KnRec<ROWS> KR;
    constexpr int NB = KR::NB;
    const long l = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (l >= nlines) return;
    auto coef = [&](int z, double (&Bz)[NB], double (&Cz)[NB]) {
        const long node = l + (long)z * nlines;
        const double v = vol[node];
        for (int e = 0; e < NB; ++e) {
            Bz[e] = rows[(long)e * nn + node];
            Cz[e] = v * Bz[e];
        }
    };
    double BL[NB], CL[NB], Bz[NB], Cz[NB];
    coef(zref, BL, CL);
    double* o = lrec + l * KR::LINE;
    for (int e = 0; e < NB; ++e) {
        o[e] = BL[e];
        o[NB + e] = CL[e];
    }
    int ci = 0;
    for (int z = 0; z < nz; ++z) {
        const bool corr = ci < nc && czl[ci] == z;
        coef(z, Bz, Cz);
        if (corr) {
            for (int e = 0; e < NB; ++e) {
                o[2 * NB + 2 * NB * ci + e] = Bz[e] - BL[e];
                o[2 * NB + 2 * NB * ci + NB + e] = Cz[e] - CL[e];
            }
            ++ci;
        } else {
            for (int e = 0; e < NB; ++e)
                if (fabs(Bz[e] - BL[e]) > tolb || fabs(Cz[e] - CL[e]) > tolc) atomicOr(bad, 1);
        }
    }
}

// Pair records: the mean and half difference of the two lines' B_L and C_L,
// the correction entries of both lines interleaved, the mismatch flag; pairs
// equal to the reference pair share record 0, as for K's records.
template <int ROWS>
__global__ void k_kn_pairs(const double* __restrict__ lrec, long npairs, int nc, long pref, double tolb,
                           double tolc, int* __restrict__ pidx, double* __restrict__ rec)
{
    typedef KnRec<ROWS> KR;
    constexpr int NB = KR::NB;
    const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const double* A = lrec + (2 * p) * KR::LINE;
    const double* B = A + KR::LINE;
    // B or C entry of a line record word
    auto tol_of = [&](int k) { return ((k < 2 * NB ? k : k - 2 * NB) % (2 * NB)) < NB ? tolb : tolc; };
    auto write = [&](double* o) {
        bool mism = false;
        for (int e = 0; e < 2 * NB; ++e) {
            const double hd = 0.5 * (A[e] - B[e]);
            const int k = e < NB ? e : NB + e;   // B mean/half at 0/NB, C mean/half at 2NB/3NB
            o[k] = 0.5 * (A[e] + B[e]);
            o[k + NB] = hd;
            mism = mism || fabs(hd) > tol_of(e);
        }
        for (int ci = 0; ci < kSymC; ++ci)
            for (int e = 0; e < 2 * NB; ++e) {
                o[KR::HEAD + KR::CORR * ci + 2 * e] = ci < nc ? A[2 * NB + 2 * NB * ci + e] : 0.0;
                o[KR::HEAD + KR::CORR * ci + 2 * e + 1] = ci < nc ? B[2 * NB + 2 * NB * ci + e] : 0.0;
            }
        for (int k = KR::HEAD + KR::CORR * kSymC; k < KR::REC; ++k) o[k] = 0.0;
        o[KR::FLAG] = mism ? 1.0 : 0.0;
    };
    bool same = pref >= 0;
    if (same) {
        const double* RA = lrec + (2 * pref) * KR::LINE;
        for (int k = 0; k < 2 * NB + 2 * NB * nc && same; ++k)
            same = fabs(A[k] - RA[k]) <= tol_of(k) && fabs(B[k] - RA[KR::LINE + k]) <= tol_of(k);
    }
    write(rec + (size_t)(1 + p) * KR::REC);
    if (p == pref) write(rec);
    pidx[p] = same ? 0 : (int)(1 + p);
}

namespace {
// builds one record set (synchronous); false where it cannot be
template <int ROWS>
bool kn_records(const Ctx& c, const double* rows, double bscale, double vscale, int*& pidx, double*& recs,
                hipStream_t st)
{
    typedef KnRec<ROWS> KR;
    const SymState& s = *(const SymState*)c.sym;
    const SymTab& tab = s.htab;
    const long nlines = (long)c.n[0] * c.n[1], npairs = nlines / 2;
    if (!(bscale > 0.0) || !(vscale > 0.0)) return false;
    const double tolb = 1e-11 * bscale, tolc = 1e-11 * bscale * vscale;
    double* lrec = nullptr;
    int* czl = nullptr;
    int* flag = nullptr;
    bool ok = sym_alloc(pidx, npairs) && sym_alloc(recs, (size_t)(npairs + 1) * KR::REC) &&
              sym_alloc(lrec, (size_t)nlines * KR::LINE) && sym_alloc(czl, kSymC) && sym_alloc(flag, 1);
    if (ok) {
        int hflag = 0;
        (void)hipMemcpyAsync(czl, tab.cz, sizeof(int) * kSymC, hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(flag, &hflag, sizeof(int), hipMemcpyHostToDevice, st);
        hipLaunchKernelGGL((k_kn_lines<ROWS>), dim3((unsigned)((nlines + 255) / 256)), dim3(256), 0, st, rows,
                           c.vol64, nlines, c.n[2], c.nn, s.zref, tab.nc, czl, tolb, tolc, lrec, flag);
        const long pref = ((long)(c.n[0] / 2) + (long)c.n[0] * (c.n[1] / 2)) / 2;
        hipLaunchKernelGGL((k_kn_pairs<ROWS>), dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, st, lrec,
                           npairs, tab.nc, pref, tolb, tolc, pidx, recs);
        (void)hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st);
        ok = hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess && hflag == 0;
    }
    (void)hipGetLastError();
    sym_free(lrec);
    sym_free(czl);
    sym_free(flag);
    if (!ok) {
        sym_free(pidx);
        sym_free(recs);
    }
    return ok;
}

// the gradient's records (rows b^a) and those of b^0, built once
bool kn_build(const Ctx& c, hipStream_t st)
{
    SymState* s = (SymState*)c.sym;
    if (s->kn != 0) return s->kn > 0;
    s->kn = -1;
    double bscale = 0.0;
    for (int e = 0; e < 12; ++e) bscale = std::max(bscale, fabs(c.nconst.b[e]));
    if (!kn_records<3>(c, c.ba_64, bscale, c.nconst.v, s->knpidx, s->knrec, st)) return false;
    // b^0 at the box centre gives its scale (interior node of a cube-like domain)
    const long centre = (long)(c.n[0] / 2) + (long)c.n[0] * ((c.n[1] / 2) + (long)c.n[1] * (c.n[2] / 2));
    double b0c[4] = {0, 0, 0, 0};
    for (int q = 0; q < 4; ++q)
        if (hipMemcpy(&b0c[q], c.b0_64 + (size_t)q * c.nn + centre, sizeof(double), hipMemcpyDeviceToHost) !=
            hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
    double b0scale = 0.0;
    for (int q = 0; q < 4; ++q) b0scale = std::max(b0scale, fabs(b0c[q]));
    if (!kn_records<1>(c, c.b0_64, b0scale, c.nconst.v, s->b0pidx, s->b0rec, st)) {
        sym_free(s->knpidx);
        sym_free(s->knrec);
        return false;
    }
    s->kn = 1;
    return true;
}

template <class Lay>
void run_kn(const Ctx& c, const double* in, double* out, double kappa, int mode, hipStream_t st)
{
    const SymState& s = *(const SymState*)c.sym;
    const long nn = c.nn;
    const long slot_rb = 2L * c.basis_plan.maxpairs * nn;
    double* S1 = reinterpret_cast<double*>(c.work64);
    double* S2 = S1 + slot_rb * c.cap_work;
    const dim3 grid((unsigned)blocks_of<Lay>(c), 1u), block(kRT);
    const RegProf prof{};
    auto args = [&](int axis, const double* i, long irb, double* o, long orb) {
        RArgsT<double> a{};
        a.in = i;
        a.in_rb = irb;
        a.out = o;
        a.out_rb = orb;
        a.fstride = nn;
        a.st = axis == 0 ? 1 : (axis == 1 ? (long)c.n[0] : (long)c.n[0] * c.n[1]);
        a.tr = c.rtab64[axis];
        a.tw = c.tw64[axis];
        return a;
    };
    const bool part1 = mode != RK_LOAD, part2 = mode == RK_FORCE || mode == RK_LOAD;
    if (part1) {
        {
            RArgsT<double> a = args(0, in, nn, S1, slot_rb);
            a.mask_in = c.chi;
            rlaunch(prof, 0, k_rpass<Lay, Lin3, 1, true, true, false, 1, 0, false, double>, grid, block, st, a);
        }
        RArgsT<double> a = args(1, S1, slot_rb, S2, slot_rb);
        rlaunch(prof, 1, k_rpass<Lay, Lin3, 1, false, false, false, 1, 1, false, double>, grid, block, st, a);
    }
    KArgs<double> k{};
    k.in = part1 ? S2 : in;
    k.in_rb = part1 ? slot_rb : nn;
    k.out = part2 ? S1 : out;
    k.out_rb = part2 ? slot_rb : nn;
    k.fstride = nn;
    k.st = (long)c.n[0] * c.n[1];
    k.tr = c.rtab64[2];
    k.tw = c.tw64[2];
    k.tab = s.tab;
    k.kappa = kappa;
    k.mask = c.chi;
    const bool b0 = mode == RK_UH || mode == RK_LOAD;
    k.pidx = b0 ? s.b0pidx : s.knpidx;
    k.rec = b0 ? s.b0rec : s.knrec;
    switch (mode) {
        case RK_FORCE: hipLaunchKernelGGL((k_smid_kn<Lay, double, KN_FORCE, 3>), grid, block, 0, st, k); break;
        case RK_GRAD: hipLaunchKernelGGL((k_smid_kn<Lay, double, KN_GRAD, 3>), grid, block, 0, st, k); break;
        case RK_UH: hipLaunchKernelGGL((k_smid_kn<Lay, double, KN_GRAD, 1>), grid, block, 0, st, k); break;
        default: hipLaunchKernelGGL((k_smid_kn<Lay, double, KN_LOAD, 1>), grid, block, 0, st, k); break;
    }
    if (!part2) return;
    {
        RArgsT<double> a = args(1, S1, slot_rb, S2, slot_rb);
        rlaunch(prof, 3, k_rpass<Lay, Lin3, 1, false, false, false, 2, 1, false, double>, grid, block, st, a);
    }
    {
        RArgsT<double> a = args(0, S2, slot_rb, out, nn);
        a.mask_out = c.chi;
        rlaunch(prof, 4, k_rpass<Lay, Lin3, 1, true, false, true, 2, 0, false, double>, grid, block, st, a);
    }
}
}  // namespace

// the FP64 register path serves the gradient nonlinearity, u^h and f^r
// (records built on first use)
bool reg_kn_ok(const Ctx& c, hipStream_t st)
{
    // K's own rows (every operator set has dim + 1 rows or one); setup builds
    // the records, so a product under graph capture never does
    if (c.krows != c.dim || !reg_path64_ok(c) || !c.sym) return false;
    if (((const SymState*)c.sym)->kn == 0 && c.capturing) return false;
    return kn_build(c, st);
}

// one field: the gradient force, the three components of the implicit
// gradient B d (out holds 3 fields), u^h, or the load f^r (mode RK_*)
void launch_reg_kn(const Ctx& c, const double* in, double* out, double kappa, int mode, hipStream_t st)
{
    if (c.n[0] == 128) run_kn<G16L>(c, in, out, kappa, mode, st);
    else if (c.n[0] == 32) run_kn<GPQ<4, 8>>(c, in, out, kappa, mode, st);
    else if (c.n[0] == 48) run_kn<GPQ<6, 8>>(c, in, out, kappa, mode, st);
    else if (c.n[0] == 80) run_kn<G16P<5>>(c, in, out, kappa, mode, st);
    else if (c.n[0] == 96) run_kn<G16P<6>>(c, in, out, kappa, mode, st);
    else if (c.n[0] == 256) run_kn<G32>(c, in, out, kappa, mode, st);
    else run_kn<G8<8>>(c, in, out, kappa, mode, st);
}

}  // namespace fcrkpm
