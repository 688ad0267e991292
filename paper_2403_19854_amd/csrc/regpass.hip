// regpass.hip -- register-resident separable passes of the FP32 stiffness
// product K d (Alg 2) on 3D boxes whose axes are 64 or 128 nodes long, for
// the linear basis.
//
// A complex line packs two adjacent real lines of one field: the real part is
// line w, the imaginary part line w+1.  Every 1D kernel array t_e is real
// (Eq 77-78), so one complex convolution convolves both lines at once and no
// spectral separation is needed; t_e is even or odd in its offset, so its
// spectrum is real or imaginary and one float per frequency describes it.
//
// A complex line of L points is owned by a group of lanes that hold it in
// registers, in one of two layouts:
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
// pointwise stage of the middle pass all act on registers.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

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
template <int DIR>
__device__ __forceinline__ cf mul_w16(cf a, int j)
{
    constexpr float C[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                             0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                             -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                             0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
    const float c = C[j & 15], s = C[(j + 12) & 15];  // sin(x) = cos(x - pi/2)
    const float ds = DIR > 0 ? s : -s;
    return cf{a.x * c + a.y * ds, a.y * c - a.x * ds};
}

// in-place DFT-16 in natural order, as 4 x 4 with internal twiddles
template <int DIR>
__device__ __forceinline__ void dft16(cf* v)
{
    cf a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
        dft4<float, DIR>(a[n2]);
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1)
            if (n2 > 0) a[n2][k1] = mul_w16<DIR>(a[n2][k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cf b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4<float, DIR>(b);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
}

template <int R, int DIR>
__device__ __forceinline__ void dftR_reg(cf* v)
{
    if constexpr (R == 16) dft16<DIR>(v);
    else dft8<float, DIR>(v);
}

template <int DIR>
__device__ __forceinline__ cf twid(const cf* tw, int j)
{
    const cf w = tw[j];
    return DIR > 0 ? w : cf{w.x, -w.y};
}

// Forward transform of the group's line.  In: v[m] = x[t + 8m].  Out:
// v[8j + k2] = X[t + 8j + R k2] (j < R/8, k2 < 8).
template <int R>
__device__ __forceinline__ void g8_fwd(cf (&v)[R], int t, cf* xb, const cf* tw)
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
    for (int j = 0; j < KPL; ++j) dft8<float, +1>(v + 8 * j);
}

// Unnormalised inverse: the layout of fwd's output in, x[t + 8m] in v[m] out.
template <int R>
__device__ __forceinline__ void g8_inv(cf (&v)[R], int t, cf* xb, const cf* tw)
{
    constexpr int KPL = R / 8;
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
        dft8<float, -1>(v + 8 * j);
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

// The twiddles one G16 lane needs, fixed for the whole kernel: the forward
// W_128^{t k1} (k1 = 1..7), the W_16^{tl h} of its half (1 on h = 0) and the
// inverse W_128^{-(tl + 8h) (t & 7)} (tl = 0..7).  Computed once per lane from
// the LDS table, so the transforms read no twiddles and select nothing.
struct G16Tw {
    cf f[7], h[7], i[8];
    __device__ __forceinline__ void make(int t, const cf* tw)
    {
        const int k1 = t & 7, hh = t >> 3;
#pragma unroll
        for (int j = 1; j < 8; ++j) {
            f[j - 1] = tw[t * j];
            const cf w = mul_w16<+1>(cf{1.0f, 0.0f}, j);
            h[j - 1] = hh ? w : cf{1.0f, 0.0f};
        }
#pragma unroll
        for (int tl = 0; tl < 8; ++tl) i[tl] = twid<-1>(tw, (tl + 8 * hh) * k1);
    }
};

// G16 forward transform (L = 128).  In: v[m] = x[t + 16m].  Out: v[i] =
// X[t + 16i].  With t = k1 + 8h the steps are a DFT-8 over m, the twiddle
// W_128^{t k1}, a transpose giving lane (k1, h) the values of lanes
// 8h .. 8h+7 at k1, a radix-2 step across h, the twiddle W_16^{tl h} and a
// DFT-8 over the lane offset tl.
__device__ __forceinline__ void g16_fwd(cf (&v)[8], int t, cf* xb, const G16Tw& w)
{
    dft8<float, +1>(v);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) v[k1] = cmul(v[k1], w.f[k1 - 1]);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) xb[k1 * 17 + t] = v[k1];
    wave_sync();
    const int k1 = t & 7, h = t >> 3;
#pragma unroll
    for (int tl = 0; tl < 8; ++tl) v[tl] = xb[k1 * 17 + 8 * h + tl];
    wave_sync();
    const float s = h ? -1.0f : 1.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const cf u = {swap8(v[i].x), swap8(v[i].y)};
        v[i] = cf{u.x + s * v[i].x, u.y + s * v[i].y};
    }
#pragma unroll
    for (int tl = 1; tl < 8; ++tl) v[tl] = cmul(v[tl], w.h[tl - 1]);
    dft8<float, +1>(v);
}

// G16 unnormalised inverse: v[i] = X[t + 16i] in, v[m] = x[t + 16m] out (the
// steps of g16_fwd reversed, with conjugate twiddles).
__device__ __forceinline__ void g16_inv(cf (&v)[8], int t, cf* xb, const G16Tw& w)
{
    const int k1 = t & 7, h = t >> 3;
    dft8<float, -1>(v);
#pragma unroll
    for (int tl = 1; tl < 8; ++tl) v[tl] = cmulc(v[tl], w.h[tl - 1]);
    const float s = h ? -1.0f : 1.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const cf u = {swap8(v[i].x), swap8(v[i].y)};
        v[i] = cf{u.x + s * v[i].x, u.y + s * v[i].y};
    }
#pragma unroll
    for (int tl = 0; tl < 8; ++tl) xb[k1 * 17 + tl + 8 * h] = cmul(v[tl], w.i[tl]);
    wave_sync();
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = xb[j * 17 + t];
    wave_sync();
    dft8<float, -1>(v);
}

// The lane's values of the axis's two kernel spectra, each divided by L (the
// 1/L of the inverse transform): T_0 is real (t_0 even) and T_1 imaginary
// (t_1 odd), so one float per frequency describes each.  G16 holds its 8
// frequencies of both in registers; G8 reads them from the LDS copy.
struct SpecRegs {
    float s0[8], s1[8];
    template <class Lay>
    __device__ __forceinline__ void fetch(const float* tab, int t)
    {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            s0[i] = tab[Lay::freq(t, i)];
            s1[i] = tab[Lay::L + Lay::freq(t, i)];
        }
    }
    template <class Lay>
    __device__ __forceinline__ void bind(const float*, int) {}
    template <class Lay>
    __device__ __forceinline__ float e0(int i) const { return s0[i]; }
    template <class Lay>
    __device__ __forceinline__ float e1(int i) const { return s1[i]; }
};
struct SpecLds {
    const float* trl;
    int t;
    template <class Lay>
    __device__ __forceinline__ void fetch(const float*, int) {}
    template <class Lay>
    __device__ __forceinline__ void bind(const float* tab, int lane)
    {
        trl = tab;
        t = lane;
    }
    template <class Lay>
    __device__ __forceinline__ float e0(int i) const { return trl[Lay::freq(t, i)]; }
    template <class Lay>
    __device__ __forceinline__ float e1(int i) const { return trl[Lay::L + Lay::freq(t, i)]; }
};

// Line layouts: lanes per complex line, points per lane, the spatial row of
// point m and the frequency of spectral slot i held by lane t, the LDS
// complex values of one group's transpose buffer (the group stride is 8 mod
// 32 so the groups of a wave spread over the banks), and the geometry of the
// staging buffer of strided passes (TP, SS, STAGE; see stage_move).
// G8 reads its twiddles from the LDS table as it goes
struct LdsTw {
    const cf* tw;
    __device__ __forceinline__ void make(int, const cf* table) { tw = table; }
};

template <int R>
struct G8 {
    static constexpr int LANES = 8, PTS = R, L = 8 * R, XS = R == 16 ? 168 : 72;
    static constexpr int GROUPS = kRT / LANES, LINES = 2 * GROUPS;
    static constexpr int TP = GROUPS + 1, SS = LANES * TP, STAGE = PTS * SS;
    typedef LdsTw Tw;
    typedef SpecLds Spec;
    static __device__ __forceinline__ int row(int t, int m) { return t + 8 * m; }
    static __device__ __forceinline__ int freq(int t, int i) { return t + 8 * (i / 8) + R * (i % 8); }
    static __device__ __forceinline__ void fwd(cf (&v)[R], int t, cf* xb, const Tw& w) { g8_fwd<R>(v, t, xb, w.tw); }
    static __device__ __forceinline__ void inv(cf (&v)[R], int t, cf* xb, const Tw& w) { g8_inv<R>(v, t, xb, w.tw); }
};
struct G16 {
    static constexpr int LANES = 16, PTS = 8, L = 128, XS = 136;
    static constexpr int GROUPS = kRT / LANES, LINES = 2 * GROUPS;
    static constexpr int TP = GROUPS + 1, SS = LANES * TP, STAGE = PTS * SS;
    typedef G16Tw Tw;
    typedef SpecRegs Spec;
    static __device__ __forceinline__ int row(int t, int m) { return t + 16 * m; }
    static __device__ __forceinline__ int freq(int t, int i) { return t + 16 * i; }
    static __device__ __forceinline__ void fwd(cf (&v)[8], int t, cf* xb, const Tw& w) { g16_fwd(v, t, xb, w); }
    static __device__ __forceinline__ void inv(cf (&v)[8], int t, cf* xb, const Tw& w) { g16_inv(v, t, xb, w); }
};

// Term structure of the K d passes for the linear basis in 3D, monomials in
// graded order (1, x, y, z).  Part 1 along axis j forms output o from input
// kP1In[j][o] with the kernel t_{kP1E[j][o]}; part 2 forms output o from input
// kP2A[j][o] with t_0 and, where kP2B[j][o] >= 0, from input kP2B[j][o] with
// the reflected t_1 (Eq 55, 77-78).  reg_path_ok checks the pass programs of
// the basis against these tables before the register path is used.
constexpr int kP1In[3][4] = {{0, 0, -1, -1}, {0, 1, 0, -1}, {0, 1, 2, 0}};
constexpr int kP1E[3][4] = {{0, 1, -1, -1}, {0, 0, 1, -1}, {0, 0, 0, 1}};
constexpr int kP2A[3][3] = {{0, -1, -1}, {0, 1, -1}, {0, 1, 2}};
constexpr int kP2B[3][3] = {{1, -1, -1}, {2, -1, -1}, {3, -1, -1}};

// Spectra of output O (in fwd's layout) from the input spectra Z.  Part 1
// (more outputs than inputs): Y = T_e Z_in.  Part 2: Y = T_0 Z_a - T_1 Z_b
// (the reflected odd kernel has the conjugate spectrum).
template <class Lay, int NIN, int NOUT, int O, int R, class Sp>
__device__ __forceinline__ void combine_o(const cf (&Z)[NIN][R], cf (&Y)[R], const Sp& sp)
{
    if constexpr (NOUT > NIN) {
        constexpr int J = NOUT - 2, IN = kP1In[J][O];
        static_assert(IN >= 0 && IN < NIN, "part-1 term");
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const cf z = Z[IN][i];
            if constexpr (kP1E[J][O] == 0) {
                const float a = sp.template e0<Lay>(i);
                Y[i] = cf{a * z.x, a * z.y};
            } else {
                const float b = sp.template e1<Lay>(i);
                Y[i] = cf{-b * z.y, b * z.x};
            }
        }
    } else {
        constexpr int J = NIN - 2, A = kP2A[J][O], B = kP2B[J][O];
        static_assert(A >= 0 && A < NIN && B < NIN, "part-2 terms");
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const float a = sp.template e0<Lay>(i);
            const cf za = Z[A][i];
            if constexpr (B >= 0) {
                const float b = sp.template e1<Lay>(i);
                const cf zb = Z[B][i];
                Y[i] = cf{a * za.x + b * zb.y, a * za.y - b * zb.x};
            } else {
                Y[i] = cf{a * za.x, a * za.y};
            }
        }
    }
}

template <class Lay, int NIN, int NOUT, int R, class Sp, int... O>
__device__ __forceinline__ void combine_sel(const cf (&Z)[NIN][R], int o, cf (&Y)[R], const Sp& sp,
                                            std::integer_sequence<int, O...>)
{
    ((o == O ? combine_o<Lay, NIN, NOUT, O>(Z, Y, sp) : void()), ...);
}

// o is constant once the caller's loop over the outputs is unrolled, so the
// selection folds away
template <class Lay, int NIN, int NOUT, int R, class Sp>
__device__ __forceinline__ void combine(const cf (&Z)[NIN][R], int o, cf (&Y)[R], const Sp& sp)
{
    combine_sel<Lay, NIN, NOUT>(Z, o, Y, sp, std::make_integer_sequence<int, NOUT>{});
}

struct RArgs {
    const float* in;          // real fields fstride apart (or the field masked by mask_in)
    const uint8_t* mask_in;
    float* out;
    const uint8_t* mask_out;  // masked single-field store (and dot), else NULL
    long fstride;             // floats between fields
    long in_rb, out_rb;       // floats between right-hand sides (blockIdx.y)
    long st;                  // element stride of the axis; 1 for x
    const float* tr;          // [2][L]: Re T_0 / L, Im T_1 / L of the axis
    const cf* tw;             // [L] e^{-2 pi i j / L}
    long nn;
    double* dot_part;         // masked store: per-workgroup partial of out . dot_with
    const float* dot_with;
    const uint2* nbits;       // middle pass, per lane: .x bit 2m+c set if node c of element
                              // m is interior, .y bit m set if element m reads a record
    const uint32_t* noff;     // middle pass: per lane, its first record
    const float4* rec;        // middle pass: records of kRec floats
    float mi[10];             // middle pass: M of the interior nodes (kSym order)
    // first x pass inside CG (PUPD): the pending direction update p = r + beta p
    // with beta = (sum of rr_part) / scal[parity], written back to `in`
    const float* rvec;
    const double* rr_part;
    int nrr;
    double* scal;
    int parity;
    const int* act;
};

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
__device__ __forceinline__ void sym4_apply(const float (&M)[10], float d0, float d1, float d2, float d3,
                                           float (&e)[4])
{
    e[0] = M[0] * d0 + M[1] * d1 + M[2] * d2 + M[3] * d3;
    e[1] = M[1] * d0 + M[4] * d1 + M[5] * d2 + M[6] * d3;
    e[2] = M[2] * d0 + M[5] * d1 + M[7] * d2 + M[8] * d3;
    e[3] = M[3] * d0 + M[6] * d1 + M[8] * d2 + M[9] * d3;
}

// Position of the workgroup's Lay::LINES real lines: for a strided axis the
// float index of line l0 at point 0 (the lines are adjacent in memory), for
// x the index of line l0's first point.
template <class Lay, bool CONTIG>
__device__ __forceinline__ long tile_base(long tile, long st)
{
    const long l0 = tile * Lay::LINES;
    if (CONTIG) return l0 * Lay::L;
    const long lo = l0 % st, hi = l0 / st;
    return lo + hi * st * Lay::L;
}

// complex element m of group g: lines (2g, 2g+1) of the tile at point row(t, m)
template <class Lay, bool CONTIG>
__device__ __forceinline__ long elem_index(long base, int g, int t, int m, long st)
{
    const int i = Lay::row(t, m);
    if (CONTIG) return base + (long)(2 * g) * Lay::L + i;
    return base + 2 * g + (long)i * st;
}

template <int L, bool CONTIG>
__device__ __forceinline__ cf load_pair(const float* p, long idx)
{
    if (CONTIG) return cf{p[idx], p[idx + L]};
    const float2 v = *reinterpret_cast<const float2*>(p + idx);
    return cf{v.x, v.y};
}

template <int L, bool CONTIG>
__device__ __forceinline__ void store_pair(float* p, long idx, cf v)
{
    if (CONTIG) {
        p[idx] = v.x;
        p[idx + L] = v.y;
    } else {
        *reinterpret_cast<float2*>(p + idx) = float2{v.x, v.y};
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
// LDS, the spectra: each thread loads its share into registers (fetch) and
// writes it to LDS later (put), so these loads and those of the input lines
// are in flight together.
template <class Lay>
struct Tables {
    static constexpr int L = Lay::L;
    static constexpr bool SPEC = std::is_same<typename Lay::Spec, SpecLds>::value;
    static constexpr int NT = (L + kRT - 1) / kRT;                    // twiddles per thread
    static constexpr int NS = SPEC ? (2 * L + kRT - 1) / kRT : 0;     // spectrum values per thread
    static constexpr int LDS_SPEC = SPEC ? 2 * L : 1;                 // floats of the LDS copy
    cf w[NT];
    float s[NS > 0 ? NS : 1];
    __device__ __forceinline__ void fetch(const RArgs& a)
    {
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            const int e = threadIdx.x + i * kRT;
            if (e < L) w[i] = a.tw[e];
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int e = threadIdx.x + i * kRT;
            if (e < 2 * L) s[i] = a.tr[e];
        }
    }
    __device__ __forceinline__ void put(cf* tw, float* trl) const
    {
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            const int e = threadIdx.x + i * kRT;
            if (e < L) tw[e] = w[i];
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int e = threadIdx.x + i * kRT;
            if (e < 2 * L) trl[e] = s[i];
        }
        __syncthreads();
    }
};

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
template <class Lay>
__device__ __forceinline__ void stage_move(cf (&v)[Lay::PTS], cf* buf, int gw, int tw, int gr, int tr)
{
#pragma unroll
    for (int m = 0; m < Lay::PTS; ++m) buf[m * Lay::SS + tw * Lay::TP + gw] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < Lay::PTS; ++m) v[m] = buf[m * Lay::SS + tr * Lay::TP + gr];
}

// One separable pass: NIN real fields -> NOUT real fields along the axis.
// LMASK: the single input is masked by mask_in.  SMASK: the single output is
// masked by mask_out and, if dot_part is set, dotted with dot_with.
// TPW tiles per workgroup: the inputs of all of them are loaded up front, so
// the later tiles' loads overlap the earlier tiles' transforms and stores.
template <class Lay, int TPW, bool CONTIG, bool LMASK, bool SMASK, int NIN, int NOUT,
          bool PUPD = false>
__global__ __launch_bounds__(kRT) void k_rpass(RArgs a)
{
    constexpr int L = Lay::L, R = Lay::PTS;
    __shared__ cf tw[L];
    __shared__ float trl[Tables<Lay>::LDS_SPEC];
    __shared__ cf xbuf[Lay::GROUPS * Lay::XS];
    __shared__ double sh[kRT / 64];
    __shared__ cf stage[CONTIG ? 1 : 2][CONTIG ? 1 : Lay::STAGE];
    const int tid = threadIdx.x, g = tid / Lay::LANES, t = tid % Lay::LANES;
    const int gc = CONTIG ? g : tid % Lay::GROUPS, tc = CONTIG ? t : tid / Lay::GROUPS;
    const long rhs = blockIdx.y;
    const float* in = a.in + rhs * a.in_rb;
    float* out = a.out + rhs * a.out_rb;
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
    Tables<Lay> tabs;
    tabs.fetch(a);
    typename Lay::Spec sp;
    sp.template fetch<Lay>(a.tr, t);

    cf Z[TPW][NIN][R];
    uint8_t mk[LMASK ? TPW : 1][LMASK ? R : 1][2];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
        for (int f = 0; f < NIN; ++f)
#pragma unroll
            for (int m = 0; m < R; ++m) {
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
            for (int m = 0; m < R; ++m)
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
            const float beta = rr_old > 0.0 ? float(rr_new / rr_old) : 0.0f;
            if (blockIdx.x == 0 && tid == 0) a.scal[rhs * kScal + 1 - a.parity] = rr_new;
#pragma unroll
            for (int tt = 0; tt < TPW; ++tt) {
                const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    const cf pv = Z[tt][0][m], rv = Rv[tt][m];
                    Z[tt][0][m] = cf{rv.x + beta * pv.x, rv.y + beta * pv.y};
                    store_pair<L, CONTIG>(const_cast<float*>(in), elem_index<Lay, CONTIG>(base, gc, tc, m, a.st),
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
            for (int m = 0; m < R; ++m) {
                const cf v = Z[tt][0][m];
                Z[tt][0][m] = cf{mk[tt][m][0] ? v.x : 0.0f, mk[tt][m][1] ? v.y : 0.0f};
            }
        }
    }
    // the masked store's mask bytes and the dot's other vector, loaded after
    // the fields (loads complete in order) so they arrive during the transforms
    uint8_t mo[SMASK ? TPW : 1][SMASK ? R : 1][2];
    float dwv[SMASK ? TPW : 1][SMASK ? R : 1][2];
    if constexpr (SMASK) {
        const float* dw = a.dot_with + rhs * a.out_rb;
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
            const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
            for (int m = 0; m < R; ++m) {
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
    typename Lay::Tw lw;
    lw.make(t, tw);
    double dacc = 0.0;
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
    const long base = tile_base<Lay, CONTIG>(tile0 + tt, a.st);
#pragma unroll
    for (int f = 0; f < NIN; ++f) {
        if constexpr (!CONTIG) stage_move<Lay>(Z[tt][f], stage[(tt * (NIN + NOUT) + f) & 1], gc, tc, g, t);
        Lay::fwd(Z[tt][f], t, xb, lw);
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        cf Y[R];
        combine<Lay, NIN, NOUT>(Z[tt], o, Y, sp);
        Lay::inv(Y, t, xb, lw);
        if constexpr (!CONTIG) stage_move<Lay>(Y, stage[(tt * (NIN + NOUT) + NIN + o) & 1], g, t, gc, tc);
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const long idx = elem_index<Lay, CONTIG>(base, gc, tc, m, a.st);
            if constexpr (SMASK) {
                const float v0 = mo[tt][m][0] ? Y[m].x : 0.0f;
                const float v1 = mo[tt][m][1] ? Y[m].y : 0.0f;
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
            if (tid == 0) a.dot_part[rhs * kRedBlocks + blockIdx.x] = s;
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
    __shared__ float trl[Tables<Lay>::LDS_SPEC];
    __shared__ cf xbuf[Lay::GROUPS * Lay::XS];
    __shared__ cf stage[2][Lay::STAGE];
    const int tid = threadIdx.x, g = tid / Lay::LANES, t = tid % Lay::LANES;
    const int gc = tid % Lay::GROUPS, tc = tid / Lay::GROUPS;
    const long rhs = blockIdx.y;
    const float* in = a.in + rhs * a.in_rb;
    float* out = a.out + rhs * a.out_rb;
    const long tile0 = xcd_tile(blockIdx.x, gridDim.x) * TPW;
    cf* xb = xbuf + g * Lay::XS;
    Tables<Lay> tabs;
    tabs.fetch(a);
    typename Lay::Spec sp;
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
        for (int q = 0; q < S; ++q) combine<Lay, NIN, S>(Z[tt], q, D[q], sp);
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
            sym4_apply(a.mi, D[0][m].x, D[1][m].x, D[2][m].x, D[3][m].x, e0);
            sym4_apply(a.mi, D[0][m].y, D[1][m].y, D[2][m].y, D[3][m].y, e1);
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
        combine<Lay, S, NOUT>(D, o, Y, sp);
        Lay::inv(Y, t, xb, lw);
        stage_move<Lay>(Y, stage[(tt * (NIN + NOUT) + NIN + o) & 1], g, t, gc, tc);
#pragma unroll
        for (int m = 0; m < R; ++m)
            store_pair<L, false>(out + o * a.fstride, elem_index<Lay, false>(base, gc, tc, m, a.st), Y[m]);
    }
    }
}

template <class Lay>
long blocks_of(const Ctx& c) { return c.nn / Lay::L / Lay::LINES; }

// launch of pass k, with the sampler's events recorded by the launch itself
template <typename K>
void rlaunch(const RegProf& prof, int k, K kern, dim3 grid, dim3 block, hipStream_t st, const RArgs& a)
{
    hipEvent_t e0, e1;
    prof.events(k, &e0, &e1);
    if (e0) hipExtLaunchKernelGGL(kern, grid, block, 0, st, e0, e1, 0, a);
    else hipLaunchKernelGGL(kern, grid, block, 0, st, a);
}

template <class Lay, int TPW>
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
        a.nn = nn;
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
            rlaunch(prof, 0, k_rpass<Lay, TPW, true, true, false, 1, 2, true>, grid, block, st, a);
        } else {
            rlaunch(prof, 0, k_rpass<Lay, TPW, true, true, false, 1, 2>, grid, block, st, a);
        }
    }
    // y: X -> XY
    {
        RArgs a = args(1, S1, slot_rb, S2, slot_rb);
        rlaunch(prof, 1, k_rpass<Lay, TPW, false, false, false, 2, 3>, grid, block, st, a);
    }
    // z: XY -> D -> E -> part-2 XY
    {
        RArgs a = args(2, S2, slot_rb, S1, slot_rb);
        a.nbits = c.nbits[c.reg_layout];
        a.noff = c.noff[c.reg_layout];
        a.rec = reinterpret_cast<const float4*>(c.nrec[c.reg_layout]);
        for (int k = 0; k < 10; ++k) a.mi[k] = c.reg_mi[k];
        rlaunch(prof, 2, k_rmid<Lay, TPW, 3, 3>, grid, block, st, a);
    }
    // y: XY -> X
    {
        RArgs a = args(1, S1, slot_rb, S2, slot_rb);
        rlaunch(prof, 3, k_rpass<Lay, TPW, false, false, false, 3, 2>, grid, block, st, a);
    }
    // x: X -> f (masked), with the optional dot partials
    {
        RArgs a = args(0, S2, slot_rb, out, nn);
        a.mask_out = mask;
        a.dot_part = dot_part;
        a.dot_with = dot_with;
        rlaunch(prof, 4, k_rpass<Lay, TPW, true, false, true, 2, 1>, grid, block, st, a);
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
// in FP64 from b^a (a-major, [3][4][nn]) and V and rounded once.
template <class Lay>
__global__ void k_rmid_recs(const uint2* __restrict__ bits, const uint32_t* __restrict__ off,
                            const double* __restrict__ ba, const double* __restrict__ vol, long st,
                            long nblk, long nn, float* __restrict__ rec)
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
                        for (int al = 0; al < 3; ++al)
                            acc += ba[(long)(al * S + p) * nn + node] * ba[(long)(al * S + q) * nn + node];
                        o[2 * sym_index(p, q) + c] = (float)(v * acc);
                    }
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
    hipLaunchKernelGGL((k_rmid_recs<Lay>), dim3(256), dim3(256), 0, st, bits, off, c.ba_64, c.vol64,
                       str, blocks_of<Lay>(c), c.nn, rec);
}

}  // namespace

// layout 0: G8 (8 lanes per line), layout 1: G16 (16 lanes, 128-point lines only)
int reg_layouts(const Ctx& c) { return c.n[0] == 128 ? 2 : 1; }

// variant v = layout + 2 (tiles - 1); 8-lane 128-point lines with 2 tiles
// per workgroup need more registers than a wave has, so that one is absent
bool reg_variant_ok(const Ctx& c, int v)
{
    if (v < 0 || v > 3 || (v & 1) >= reg_layouts(c)) return false;
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

int reg_record_floats() { return kRec; }

bool reg_path_ok(const Ctx& c)
{
    if (c.dim != 3 || c.degree != 1 || c.naxes != 3 || c.s != 4) return false;
    const SepPlan& sp = c.basis_plan;
    if (sp.size[0] != 2 || sp.size[1] != 3 || sp.size[2] != 4) return false;
    for (int j = 0; j < 3; ++j) {
        if (sp.p1[j].nin != (j == 0 ? 1 : sp.size[j - 1]) || sp.p1[j].nout != sp.size[j]) return false;
        if (sp.p2[j].nin != sp.size[j] || sp.p2[j].nout != (j == 0 ? 1 : sp.size[j - 1])) return false;
    }
    const int L = c.n[0];
    if (L != 64 && L != 128) return false;
    if (c.n[1] != L || c.n[2] != L) return false;
    // the kernels hard-wire the terms of the passes (kP1In .. kP2B) and the
    // coefficient +-1/(2L) of every term
    for (int j = 0; j < 3; ++j) {
        if (c.axes[j] != j) return false;
        const double inv = 1.0 / (2.0 * c.n[j]);
        const SepProg& f = sp.p1[j];
        for (int o = 0; o < f.nout; ++o) {
            if (f.ostart[o + 1] - f.ostart[o] != 1) return false;
            const SepTerm& tm = f.t[f.ostart[o]];
            if (tm.in != kP1In[j][o] || tm.e != kP1E[j][o] || tm.coef != inv) return false;
        }
        const SepProg& g = sp.p2[j];
        for (int o = 0; o < g.nout; ++o) {
            const int nt = g.ostart[o + 1] - g.ostart[o];
            if (nt != (kP2B[j][o] >= 0 ? 2 : 1)) return false;
            for (int k = g.ostart[o]; k < g.ostart[o + 1]; ++k) {
                const SepTerm& tm = g.t[k];
                const bool ok0 = tm.e == 0 && tm.in == kP2A[j][o] && tm.coef == inv;
                const bool ok1 = tm.e == 1 && tm.in == kP2B[j][o] && tm.coef == -inv;
                if (!ok0 && !ok1) return false;
            }
        }
    }
    return true;
}

// workgroups of one launch (each covers reg_tpw tiles)
int reg_path_blocks(const Ctx& c)
{
    long b;
    if (c.n[0] == 128) b = c.reg_layout ? blocks_of<G16>(c) : blocks_of<G8<16>>(c);
    else b = blocks_of<G8<8>>(c);
    return (int)(b / c.reg_tpw);
}

void launch_reg_k(const Ctx& c, const float* in, float* out, const uint8_t* mask, int nrhs,
                  double* dot_part, const float* dot_with, hipStream_t st, const RegProf& prof,
                  const RegPupd* pu)
{
#define FC_RUN(LAY)                                                                       \
    do {                                                                                  \
        if (c.reg_tpw == 2) run_k<LAY, 2>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu); \
        else run_k<LAY, 1>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu);        \
    } while (0)
    if (c.n[0] == 128) {
        if (c.reg_layout) FC_RUN(G16);
        else run_k<G8<16>, 1>(c, in, out, mask, nrhs, dot_part, dot_with, st, prof, pu);  // 2 tiles spill
    } else {
        FC_RUN(G8<8>);
    }
#undef FC_RUN
}

}  // namespace fcrkpm
