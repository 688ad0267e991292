// fft_core.hpp -- device building blocks of the gfx950 FFT: complex arithmetic,
// small-radix DFT butterflies and a Stockham autosort line transform that runs
// a tile of W lines held in LDS.
//
// DFT convention (Sec 3, Eq 30-31): forward X_k = sum_j x_j e^{-2 pi i jk/N};
// the inverse is computed without the 1/N (callers fold 1/N into the spectral
// factors that precede every inverse transform).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcrkpm {

template <typename T>
struct cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b)  // a * conj(b)
{
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> scal(cplx<T> a, T s) { return {a.x * s, a.y * s}; }

// multiply by -i (DIR = +1, forward sign) or by +i (DIR = -1, inverse sign)
template <typename T, int DIR>
__device__ __forceinline__ cplx<T> rot90(cplx<T> a)
{
    if (DIR > 0) return {a.y, -a.x};
    return {-a.y, a.x};
}

// ------------------------------------------------------------------ butterflies
// In-place DFT of R points: v[q] <- sum_r v[r] e^{-DIR 2 pi i r q / R}.

template <typename T, int DIR>
__device__ __forceinline__ void dft2(cplx<T>* v)
{
    cplx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <typename T, int DIR>
__device__ __forceinline__ void dft3(cplx<T>* v)
{
    const T s = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
    cplx<T> t1 = v[1] + v[2], t2 = v[1] - v[2];
    cplx<T> m = {v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y};
    cplx<T> n = rot90<T, DIR>(scal(t2, s));
    v[0] = v[0] + t1;
    v[1] = m + n;
    v[2] = m - n;
}

template <typename T, int DIR>
__device__ __forceinline__ void dft4(cplx<T>* v)
{
    cplx<T> a0 = v[0] + v[2], a1 = v[0] - v[2];
    cplx<T> a2 = v[1] + v[3], a3 = rot90<T, DIR>(v[1] - v[3]);
    v[0] = a0 + a2;
    v[2] = a0 - a2;
    v[1] = a1 + a3;
    v[3] = a1 - a3;
}

template <typename T, int DIR>
__device__ __forceinline__ void dft5(cplx<T>* v)
{
    const T c1 = T(0.30901699437494742410229341718282);   // cos(2 pi / 5)
    const T c2 = T(-0.80901699437494742410229341718282);  // cos(4 pi / 5)
    const T s1 = T(0.95105651629515357211643933337938);   // sin(2 pi / 5)
    const T s2 = T(0.58778525229247312916870595463907);   // sin(4 pi / 5)
    cplx<T> t1 = v[1] + v[4], t2 = v[2] + v[3];
    cplx<T> t3 = v[1] - v[4], t4 = v[2] - v[3];
    cplx<T> a1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    cplx<T> a2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    cplx<T> b1 = rot90<T, DIR>(cplx<T>{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
    cplx<T> b2 = rot90<T, DIR>(cplx<T>{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
    v[0] = v[0] + t1 + t2;
    v[1] = a1 + b1;
    v[4] = a1 - b1;
    v[2] = a2 + b2;
    v[3] = a2 - b2;
}

// seven points: conjugate-symmetric pairs t_k = v_k + v_(7-k), u_k = v_k - v_(7-k)
template <typename T, int DIR>
__device__ __forceinline__ void dft7(cplx<T>* v)
{
    const T c1 = T(0.62348980185873353052500488400424);   // cos(2 pi / 7)
    const T c2 = T(-0.22252093395631440428890256449679);  // cos(4 pi / 7)
    const T c3 = T(-0.90096886790241912623610231950745);  // cos(6 pi / 7)
    const T s1 = T(0.78183148246802980870844452667406);   // sin(2 pi / 7)
    const T s2 = T(0.97492791218182360701813168299393);   // sin(4 pi / 7)
    const T s3 = T(0.43388373911755812047576833284836);   // sin(6 pi / 7)
    const cplx<T> t1 = v[1] + v[6], t2 = v[2] + v[5], t3 = v[3] + v[4];
    const cplx<T> u1 = v[1] - v[6], u2 = v[2] - v[5], u3 = v[3] - v[4];
    const cplx<T> a1 = {v[0].x + c1 * t1.x + c2 * t2.x + c3 * t3.x, v[0].y + c1 * t1.y + c2 * t2.y + c3 * t3.y};
    const cplx<T> a2 = {v[0].x + c2 * t1.x + c3 * t2.x + c1 * t3.x, v[0].y + c2 * t1.y + c3 * t2.y + c1 * t3.y};
    const cplx<T> a3 = {v[0].x + c3 * t1.x + c1 * t2.x + c2 * t3.x, v[0].y + c3 * t1.y + c1 * t2.y + c2 * t3.y};
    const cplx<T> b1 = rot90<T, DIR>(cplx<T>{s1 * u1.x + s2 * u2.x + s3 * u3.x, s1 * u1.y + s2 * u2.y + s3 * u3.y});
    const cplx<T> b2 = rot90<T, DIR>(cplx<T>{s2 * u1.x - s3 * u2.x - s1 * u3.x, s2 * u1.y - s3 * u2.y - s1 * u3.y});
    const cplx<T> b3 = rot90<T, DIR>(cplx<T>{s3 * u1.x - s1 * u2.x + s2 * u3.x, s3 * u1.y - s1 * u2.y + s2 * u3.y});
    v[0] = v[0] + t1 + t2 + t3;
    v[1] = a1 + b1;
    v[6] = a1 - b1;
    v[2] = a2 + b2;
    v[5] = a2 - b2;
    v[3] = a3 + b3;
    v[4] = a3 - b3;
}

template <typename T, int DIR>
__device__ __forceinline__ void dft8(cplx<T>* v)
{
    const T r = T(0.70710678118654752440084436210485);  // 1 / sqrt(2)
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T, DIR>(e);
    dft4<T, DIR>(o);
    // o[q] *= w^q with w = e^{-DIR 2 pi i / 8}
    cplx<T> o1, o3;
    if (DIR > 0) {
        o1 = {r * (o[1].x + o[1].y), r * (o[1].y - o[1].x)};
        o3 = {r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y)};
    } else {
        o1 = {r * (o[1].x - o[1].y), r * (o[1].x + o[1].y)};
        o3 = {-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y)};
    }
    cplx<T> o2 = rot90<T, DIR>(o[2]);
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
}

template <typename T, int DIR, int R>
__device__ __forceinline__ void dftR(cplx<T>* v)
{
    if constexpr (R == 2) dft2<T, DIR>(v);
    else if constexpr (R == 3) dft3<T, DIR>(v);
    else if constexpr (R == 4) dft4<T, DIR>(v);
    else if constexpr (R == 5) dft5<T, DIR>(v);
    else if constexpr (R == 7) dft7<T, DIR>(v);
    else dft8<T, DIR>(v);
}

// ----------------------------------------------------------------- line plans

constexpr int kMaxStages = 12;

// Radix factorisation of one axis length (product of rad[] == n).
struct LinePlan {
    int n;
    int nst;
    int rad[kMaxStages];
};

// One Stockham stage of radix R over W lines in LDS.
// Element (w, i) of a buffer sits at buf[w * sw + i * si].
// CONTIG selects the butterfly-to-thread order: lines contiguous in LDS
// (x axis, consecutive threads walk j) or interleaved (consecutive threads
// walk w).  tw[k] = e^{-2 pi i k / n}.
template <typename T, int DIR, int R, bool CONTIG>
__device__ __forceinline__ void stockham_stage(const cplx<T>* __restrict__ src,
                                               cplx<T>* __restrict__ dst, int n, int Ns, int W,
                                               int sw, int si, const cplx<T>* __restrict__ tw,
                                               int tid, int nthr)
{
    const int nb = n / R;
    const int tot = W * nb;
    const int twstep = n / (Ns * R);
    for (int b = tid; b < tot; b += nthr) {
        int w, j;
        if (CONTIG) {
            w = b / nb;
            j = b - w * nb;
        } else {
            j = b / W;
            w = b - j * W;
        }
        const int k = j % Ns;
        cplx<T> v[R];
        const cplx<T>* s = src + w * sw;
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = s[(j + r * nb) * si];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cplx<T> t = tw[k * r * twstep];
                v[r] = (DIR > 0) ? cmul(v[r], t) : cmulc(v[r], t);
            }
        }
        dftR<T, DIR, R>(v);
        const int base = (j / Ns) * Ns * R + k;
        cplx<T>* d = dst + w * sw;
#pragma unroll
        for (int r = 0; r < R; ++r) d[(base + r * Ns) * si] = v[r];
    }
}

// All stages of a length-n transform on W lines; ping-pongs between a and b
// and returns the buffer that holds the result.  Ends with a barrier.
template <typename T, int DIR, bool CONTIG>
__device__ cplx<T>* line_fft(cplx<T>* a, cplx<T>* b, const LinePlan& p, int W, int sw, int si,
                             const cplx<T>* __restrict__ tw, int tid, int nthr)
{
    int Ns = 1;
    for (int st = 0; st < p.nst; ++st) {
        const int R = p.rad[st];
        switch (R) {
            case 2: stockham_stage<T, DIR, 2, CONTIG>(a, b, p.n, Ns, W, sw, si, tw, tid, nthr); break;
            case 3: stockham_stage<T, DIR, 3, CONTIG>(a, b, p.n, Ns, W, sw, si, tw, tid, nthr); break;
            case 4: stockham_stage<T, DIR, 4, CONTIG>(a, b, p.n, Ns, W, sw, si, tw, tid, nthr); break;
            case 5: stockham_stage<T, DIR, 5, CONTIG>(a, b, p.n, Ns, W, sw, si, tw, tid, nthr); break;
            case 7: stockham_stage<T, DIR, 7, CONTIG>(a, b, p.n, Ns, W, sw, si, tw, tid, nthr); break;
            default: stockham_stage<T, DIR, 8, CONTIG>(a, b, p.n, Ns, W, sw, si, tw, tid, nthr); break;
        }
        __syncthreads();
        cplx<T>* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

}  // namespace fcrkpm
