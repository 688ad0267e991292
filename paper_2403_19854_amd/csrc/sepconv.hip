// sepconv.hip -- separable FFT convolutions along one axis at a time.
//
// The kernel of the method is a tensor product (Sec 2.1, Eq 6) and every
// convolving array is a monomial times that kernel (Eq 44, 77-79), so each 3D
// spectrum is a product of 1D spectra, F(H) = Tx(kx) Ty(ky) Tz(kz).  The 3D
// circular convolution F^-1[F(u) F(H)] (Sec 3, Eq 34) therefore factors into
// commuting 1D FFT convolutions, one per axis.  Applied as a tree over the
// monomial exponents this evaluates every convolution of Alg 1-4 with one
// pass over HBM per axis:
//
//   part 1 (Eq 90, 94):  u -> X_ax -> XY_(ax,ay) -> D_q = u (*) H_q^a
//   part 2 (Eq 91, 92):  E_p -> Z_(ax,ay) -> Y_ax -> sum_p E_p (*) Hbar_p^a
//
// A pass loads W lines of the tile into LDS, runs a forward Stockham FFT per
// pair of real fields (two real fields share one complex line), forms every
// output spectrum as a sum of input spectra times 1D kernel spectra (the
// spectrum of each real field is separated from its pair with the conjugate-
// mirror identity), and runs one inverse FFT per pair of real outputs.  The
// last axis of K d is one "middle" pass that also applies the pointwise stage
// (A^a, C_p^a of Alg 2) between the two halves, so D_q and E_p never reach HBM.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

#include "fcrkpm_impl.hpp"

namespace fcrkpm {

// ------------------------------------------------------------- tile geometry
// A workgroup owns W lines (W a power of two) of length L along the axis and
// keeps them line-contiguous in LDS with pitch L+1.  Loads, stores and the
// pointwise stage use the cooperative mapping (consecutive threads touch
// consecutive global addresses); FFT stages and spectral combinations run
// wave-locally when W is a multiple of the 4 waves (each wave owns W/4 whole
// lines), otherwise the whole workgroup cooperates.  LC > 0 fixes L at
// compile time (the hot sizes), LC = 0 reads it at run time.
constexpr int kThreads = 256;
constexpr int kWave = 64;
constexpr int kMaxTile = 2048;
constexpr int kLoadChunk = 8;   // tile elements per thread whose loads are in flight together
constexpr int kPwChunk = 4;     // the same for the pointwise stage (more loads per element)

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that each
// XCD walks a contiguous run of tiles and neighbouring tiles share its L2.
__device__ __forceinline__ long xcd_tile(long b, long nblocks)
{
    if (nblocks % 8 != 0) return b;
    return (b & 7) * (nblocks >> 3) + (b >> 3);
}

template <bool CONTIG, int LC>
struct Tile {
    long gbase;
    long st;
    int W, wl, L, P;
    __device__ __forceinline__ Tile(const AxisGeom& g, long t)
    {
        W = g.W;
        wl = g.wl;
        L = LC > 0 ? LC : g.L;
        P = L + 1;
        st = g.st;
        if (CONTIG) {
            gbase = t * (long)W * L;
        } else {
            long l0 = t * W;
            long lo = l0 % g.st, hi = l0 / g.st;
            gbase = lo + hi * g.st * L;
        }
    }
    __device__ __forceinline__ int elems() const { return W * L; }
    __device__ __forceinline__ int buf_elems() const { return W * P; }
    // cooperative mapping of tile element e: line w, position i, global gi, LDS o
    __device__ __forceinline__ void at(int e, int& w, int& i, long& gi, int& o) const
    {
        if (CONTIG) {
            w = e / L;
            i = e - w * L;
            gi = gbase + e;
        } else {
            i = e >> wl;
            w = e & (W - 1);
            gi = gbase + w + (long)i * st;
        }
        o = w * P + i;
    }
};

// The lines one wave (or the whole workgroup) works on in the local phases.
struct Crew {
    int w0, nl;    // first line and line count
    int id, n;     // thread id within the crew and crew size
    bool wave;     // wave-local (true) or workgroup-wide
};

__device__ __forceinline__ Crew make_crew(int W, int tid)
{
    Crew c;
    c.wave = (W % 4) == 0;
    if (c.wave) {
        c.nl = W / 4;
        c.w0 = (tid / kWave) * c.nl;
        c.id = tid % kWave;
        c.n = kWave;
    } else {
        c.nl = W;
        c.w0 = 0;
        c.id = tid;
        c.n = kThreads;
    }
    return c;
}

// Orders LDS accesses of the crew: a wave runs in lockstep, so a wave-scope
// fence and scheduling barrier suffice; otherwise a workgroup barrier.
__device__ __forceinline__ void crew_sync(const Crew& c)
{
    if (c.wave) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// --------------------------------------------------------------- in-place FFT
// Stockham stages done in place on the crew's lines: every thread loads the
// inputs of its butterflies, the crew synchronises, then the outputs are
// written.  A crew holds at most 8 elements per thread (W*L <= 2048 over
// 256 threads, or W/4 lines over one wave).  twl is the LDS copy of
// e^{-2 pi i k / L}, k < L.
template <int R>
constexpr int kmax_of() { return (8 + R - 1) / R; }

template <typename T, int DIR, int R, int NSC>
__device__ __forceinline__ void stage(cplx<T>* buf, int L, int P, const Crew& cr, int Ns_rt,
                                      const cplx<T>* __restrict__ twl)
{
    constexpr int KM = kmax_of<R>();
    const int Ns = (NSC > 0) ? NSC : Ns_rt;
    const int nb = L / R;
    const int tot = cr.nl * nb;
    const int twstep = L / (Ns * R);
    cplx<T> v[KM][R];
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) {
        const int b = cr.id + kk * cr.n;
        if (b < tot) {
            const int wl = b / nb, j = b - wl * nb;
            const cplx<T>* s = buf + (cr.w0 + wl) * P + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[kk][r] = s[r * nb];
        }
    }
    crew_sync(cr);
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) {
        const int b = cr.id + kk * cr.n;
        if (b < tot) {
            const int wl = b / nb, j = b - wl * nb;
            const int k = j % Ns;
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cplx<T> t = twl[k * r * twstep];
                    v[kk][r] = (DIR > 0) ? cmul(v[kk][r], t) : cmulc(v[kk][r], t);
                }
            }
            dftR<T, DIR, R>(v[kk]);
            cplx<T>* d = buf + (cr.w0 + wl) * P + (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) d[r * Ns] = v[kk][r];
        }
    }
    crew_sync(cr);
}

// radix plan of a compile-time length: 8s first, then 4s, 2, 3, 5, 7
struct CPlan {
    int nst;
    int rad[12];
};
constexpr CPlan cplan(int n)
{
    CPlan p{0, {}};
    int r = n, p2 = 0;
    while (r % 2 == 0) {
        r /= 2;
        ++p2;
    }
    int n8 = p2 / 3, rem = p2 % 3, n4 = 0, n2 = 0;
    if (rem == 2) n4 = 1;
    if (rem == 1) {
        if (n8 > 0) {
            --n8;
            n4 = 2;
        } else {
            n2 = 1;
        }
    }
    for (int i = 0; i < n8; ++i) p.rad[p.nst++] = 8;
    for (int i = 0; i < n4; ++i) p.rad[p.nst++] = 4;
    for (int i = 0; i < n2; ++i) p.rad[p.nst++] = 2;
    while (r % 3 == 0) {
        r /= 3;
        p.rad[p.nst++] = 3;
    }
    while (r % 5 == 0) {
        r /= 5;
        p.rad[p.nst++] = 5;
    }
    while (r % 7 == 0) {
        r /= 7;
        p.rad[p.nst++] = 7;
    }
    return p;
}

template <typename T, int DIR, int LC, int ST, int NS>
__device__ __forceinline__ void fft_ct(cplx<T>* buf, int P, const Crew& cr,
                                       const cplx<T>* __restrict__ twl)
{
    constexpr CPlan PL = cplan(LC);
    if constexpr (ST < PL.nst) {
        constexpr int R = PL.rad[ST];
        stage<T, DIR, R, NS>(buf, LC, P, cr, NS, twl);
        fft_ct<T, DIR, LC, ST + 1, NS * R>(buf, P, cr, twl);
    }
}

// forward (DIR=+1) or unnormalised inverse (DIR=-1) transform of the crew's lines
template <typename T, int DIR, int LC>
__device__ void fft_line(cplx<T>* buf, const LinePlan& p, int L, int P, const Crew& cr,
                         const cplx<T>* __restrict__ twl)
{
    if constexpr (LC > 0) {
        fft_ct<T, DIR, LC, 0, 1>(buf, P, cr, twl);
    } else {
        int Ns = 1;
        for (int s = 0; s < p.nst; ++s) {
            const int R = p.rad[s];
            switch (R) {
                case 2: stage<T, DIR, 2, 0>(buf, L, P, cr, Ns, twl); break;
                case 3: stage<T, DIR, 3, 0>(buf, L, P, cr, Ns, twl); break;
                case 4: stage<T, DIR, 4, 0>(buf, L, P, cr, Ns, twl); break;
                case 5: stage<T, DIR, 5, 0>(buf, L, P, cr, Ns, twl); break;
                case 7: stage<T, DIR, 7, 0>(buf, L, P, cr, Ns, twl); break;
                default: stage<T, DIR, 8, 0>(buf, L, P, cr, Ns, twl); break;
            }
            Ns *= R;
        }
    }
}

// spectrum of real field `f` (component f&1 of pair buffer f>>1) at one element
template <typename T>
__device__ __forceinline__ cplx<T> real_spec(const cplx<T>* pb, int comp, int o, int om)
{
    cplx<T> z = pb[o], zm = pb[om];
    // comp 0: (z + conj zm); comp 1: -i (z - conj zm); the 1/2 is in the term coefficient
    if (comp == 0) return cplx<T>{z.x + zm.x, z.y - zm.y};
    return cplx<T>{z.y + zm.y, zm.x - z.x};
}

// Output pair j spectrum at one element: sum over the terms of outputs 2j, 2j+1.
template <typename T>
__device__ __forceinline__ cplx<T> combine(const SepProg& pr, int j, const cplx<T>* inbase,
                                           int bstride, const cplx<T>* tab, int L, int i, int o,
                                           int om)
{
    cplx<T> acc = {T(0), T(0)};
    const int o0 = 2 * j;
#pragma unroll 1
    for (int q = 0; q < 2; ++q) {
        const int of = o0 + q;
        if (of >= pr.nout) break;
        cplx<T> part = {T(0), T(0)};
        for (int t = pr.ostart[of]; t < pr.ostart[of + 1]; ++t) {
            const SepTerm tm = pr.t[t];
            cplx<T> f = real_spec(inbase + (tm.in >> 1) * bstride, tm.in & 1, o, om);
            cplx<T> h = tab[tm.e * L + i];
            cplx<T> v = cmul(f, h);
            const T cf = T(tm.coef);
            part.x += cf * v.x;
            part.y += cf * v.y;
        }
        if (q == 0) acc = part;
        else acc = cplx<T>{acc.x - part.y, acc.y + part.x};  // + i * part
    }
    return acc;
}

// out_buf <- spectrum of output pair j for the crew's lines
template <typename T>
__device__ __forceinline__ void combine_lines(const SepProg& pr, int j, const cplx<T>* in, int BE,
                                              const cplx<T>* tab, int L, int P, const Crew& cr,
                                              cplx<T>* out_buf)
{
    const int tot = cr.nl * L;
    for (int e = cr.id; e < tot; e += cr.n) {
        const int wl = e / L, i = e - wl * L;
        const int w = cr.w0 + wl;
        const int o = w * P + i;
        const int om = w * P + (i == 0 ? 0 : L - i);
        out_buf[o] = combine<T>(pr, j, in, BE, tab, L, i, o, om);
    }
}

// ------------------------------------------------------------ generic pass
template <typename T>
struct SepArgs {
    const void* in;           // pair fields, or a real field / mask (load mode)
    const uint8_t* mask_in;
    void* out;                // pair fields, or a real field (store mode)
    const uint8_t* mask_out;
    long fstride;             // elements between consecutive pair fields
    AxisGeom g;
    LinePlan p;
    const cplx<T>* tw;
    const cplx<T>* tab;       // 1D kernel spectra of the axis, exponent-major
    int ne;                   // exponents in tab
    const SepProg* pr;        // pass program in device memory
    int nin, nout;            // its field counts
    double* dot_part;         // optional: per-block partial of out . dot_with (ST_REAL)
    const void* dot_with;
    long in_rb, out_rb;       // bytes between right-hand sides (blockIdx.y) of in / out
};

// the arguments of right-hand side blockIdx.y
template <typename T>
__device__ __forceinline__ SepArgs<T> rhs_args(const SepArgs<T>& a0)
{
    SepArgs<T> a = a0;
    const long j = blockIdx.y;
    a.in = (const char*)a0.in + j * a0.in_rb;
    a.out = (char*)a0.out + j * a0.out_rb;
    if (a0.dot_part) {
        a.dot_part = a0.dot_part + j * gridDim.x;
        a.dot_with = (const char*)a0.dot_with + j * a0.out_rb;
    }
    return a;
}

enum { LD_PAIRS = SEP_LD_PAIRS, LD_REAL = SEP_LD_REAL, LD_CHI = SEP_LD_CHI };
enum { ST_PAIRS = SEP_ST_PAIRS, ST_REAL = SEP_ST_REAL };

template <typename T, typename Tio, int LDM>
__device__ __forceinline__ cplx<T> load_elem(const SepArgs<T>& a, int bi, long gi)
{
    if constexpr (LDM == LD_PAIRS) {
        return reinterpret_cast<const cplx<T>*>(a.in)[bi * a.fstride + gi];
    } else if constexpr (LDM == LD_REAL) {
        // both loads issue together; the mask only selects
        const uint8_t mk = a.mask_in[gi];
        const T x = T(reinterpret_cast<const Tio*>(a.in)[gi]);
        return cplx<T>{mk ? x : T(0), T(0)};
    } else {
        return cplx<T>{a.mask_in[gi] ? T(1) : T(0), T(0)};
    }
}

__device__ __forceinline__ double block_reduce(double v, double* sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) r += sh[i];
    return r;
}

// cooperative load of nb pair buffers of the tile
template <typename T, typename Tio, bool CONTIG, int LDM, int LC>
__device__ __forceinline__ void load_tile(const SepArgs<T>& a, const Tile<CONTIG, LC>& tl, int nb,
                                          cplx<T>* in, int BE, int tid)
{
    // All loads of a chunk are issued before the first LDS write.  Lanes past
    // the tile end repeat its last element, which writes the same value twice.
    const int E = tl.elems();
    for (int bi = 0; bi < nb; ++bi)
        for (int base = 0; base < E; base += kLoadChunk * kThreads) {
            cplx<T> v[kLoadChunk];
            int o[kLoadChunk];
#pragma unroll
            for (int kk = 0; kk < kLoadChunk; ++kk) {
                const int e = min(base + tid + kk * kThreads, E - 1);
                int w, i;
                long gi;
                tl.at(e, w, i, gi, o[kk]);
                v[kk] = load_elem<T, Tio, LDM>(a, bi, gi);
            }
#pragma unroll
            for (int kk = 0; kk < kLoadChunk; ++kk) in[bi * BE + o[kk]] = v[kk];
        }
}

// cooperative store of one output pair; returns this thread's dot partial
template <typename T, typename Tio, bool CONTIG, int STM, int LC>
__device__ __forceinline__ double store_tile(const SepArgs<T>& a, const Tile<CONTIG, LC>& tl, int j,
                                             const cplx<T>* src, int tid)
{
    const int E = tl.elems();
    double dacc = 0.0;
    if constexpr (STM == ST_PAIRS) {
        for (int e = tid; e < E; e += kThreads) {
            int w, i, o;
            long gi;
            tl.at(e, w, i, gi, o);
            reinterpret_cast<cplx<T>*>(a.out)[j * a.fstride + gi] = src[o];
        }
    } else {
        // masks (and the dot operand) of a chunk are loaded before any store
        const bool dot = a.dot_part != nullptr;
        for (int base = 0; base < E; base += kLoadChunk * kThreads) {
            uint8_t mk[kLoadChunk];
            Tio dw[kLoadChunk];
            long g[kLoadChunk];
            int o[kLoadChunk];
#pragma unroll
            for (int kk = 0; kk < kLoadChunk; ++kk) {
                const int e = min(base + tid + kk * kThreads, E - 1);
                int w, i;
                tl.at(e, w, i, g[kk], o[kk]);
                mk[kk] = a.mask_out[g[kk]];
                dw[kk] = dot ? reinterpret_cast<const Tio*>(a.dot_with)[g[kk]] : Tio(0);
            }
#pragma unroll
            for (int kk = 0; kk < kLoadChunk; ++kk) {
                if (base + tid + kk * kThreads < E) {
                    const Tio v = mk[kk] ? Tio(src[o[kk]].x) : Tio(0);
                    reinterpret_cast<Tio*>(a.out)[g[kk]] = v;
                    dacc += (double)v * (double)dw[kk];
                }
            }
        }
    }
    return dacc;
}

template <typename T, typename Tio, bool CONTIG, int LDM, int STM, int LC>
__global__ __launch_bounds__(kThreads) void k_sep_pass(SepArgs<T> a0)
{
    const SepArgs<T> a = rhs_args(a0);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Tile<CONTIG, LC> tl(a.g, xcd_tile(blockIdx.x, gridDim.x));
    const int tid = threadIdx.x;
    const int L = tl.L, P = tl.P, BE = tl.buf_elems();
    const int nbin = (a.nin + 1) / 2, nbout = (a.nout + 1) / 2;
    const SepProg& pr = *a.pr;
    cplx<T>* tab = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* twl = tab + a.ne * L;
    cplx<T>* in = twl + L;
    cplx<T>* work = in + nbin * BE;
    for (int e = tid; e < a.ne * L; e += kThreads) tab[e] = a.tab[e];
    for (int e = tid; e < L; e += kThreads) twl[e] = a.tw[e];
    load_tile<T, Tio, CONTIG, LDM, LC>(a, tl, nbin, in, BE, tid);
    __syncthreads();
    const Crew cr = make_crew(tl.W, tid);
    for (int bi = 0; bi < nbin; ++bi) fft_line<T, +1, LC>(in + bi * BE, a.p, L, P, cr, twl);
    double dacc = 0.0;
    for (int j = 0; j < nbout; ++j) {
        combine_lines<T>(pr, j, in, BE, tab, L, P, cr, work);
        crew_sync(cr);
        fft_line<T, -1, LC>(work, a.p, L, P, cr, twl);
        __syncthreads();
        dacc += store_tile<T, Tio, CONTIG, STM, LC>(a, tl, j, work, tid);
        __syncthreads();
    }
    if constexpr (STM == ST_REAL) {
        if (a.dot_part) {
            __shared__ double sh[kThreads / 64];
            double s = block_reduce(dacc, sh);
            if (tid == 0) a.dot_part[blockIdx.x] = s;
        }
    }
}

// ------------------------------------------------------------- middle pass
// Last axis: part-1 outputs D_q stay in LDS, the pointwise stage runs per
// node, and the part-2 convolutions start from the LDS copy.
template <typename T>
struct MidArgs {
    SepArgs<T> s;             // in / out / geometry / part-1 program in s.pr
    const SepProg* pr2;       // part-2 program (E_p -> outputs), device memory
    int nout2;
    const T* b0;              // [s][nn]
    const T* ba;              // [dim][s][nn]
    const T* vol;             // [nn] or NULL
    const uint8_t* cls;       // PW_K: node class (0 outside, 1 interior, 2 other) or NULL
    T cint[kMaxNodeConst + 1];  // PW_K: b^a (a-major) and V of the interior nodes
    T kappa;                  // PW_KN: A^a -> (1 + kappa |A|^2) A^a
    const void* src;          // PW_LOAD: the real field r (Tio)
    long nn;
    long src_rb;              // bytes between right-hand sides of src
};

enum { PW_K = SEP_PW_K, PW_UH = SEP_PW_UH, PW_LOAD = SEP_PW_LOAD, PW_KN = SEP_PW_KN };

template <typename T, typename Tio, bool CONTIG, int LDM, int STM, int S, int DIM, int PW, int LC>
__global__ __launch_bounds__(kThreads) void k_sep_mid(MidArgs<T> m)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SepArgs<T> a = rhs_args(m.s);
    const void* const msrc = (const char*)m.src + (long)blockIdx.y * m.src_rb;
    const Tile<CONTIG, LC> tl(a.g, xcd_tile(blockIdx.x, gridDim.x));
    const int tid = threadIdx.x;
    const int L = tl.L, P = tl.P, E = tl.elems(), BE = tl.buf_elems();
    constexpr int NP = (S + 1) / 2;  // pair buffers of D_q / E_p
    const int nbin = (PW == PW_LOAD) ? 0 : (a.nin + 1) / 2;
    cplx<T>* tab = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* twl = tab + a.ne * L;
    cplx<T>* in = twl + L;
    cplx<T>* dbuf = in + nbin * BE;
    cplx<T>* work = dbuf + NP * BE;
    for (int e = tid; e < a.ne * L; e += kThreads) tab[e] = a.tab[e];
    for (int e = tid; e < L; e += kThreads) twl[e] = a.tw[e];
    const Crew cr = make_crew(tl.W, tid);

    if constexpr (PW != PW_LOAD) {
        load_tile<T, Tio, CONTIG, LDM, LC>(a, tl, nbin, in, BE, tid);
        __syncthreads();
        for (int bi = 0; bi < nbin; ++bi) fft_line<T, +1, LC>(in + bi * BE, a.p, L, P, cr, twl);
        // D_q (pairs) into dbuf
        const SepProg& pr1 = *a.pr;
        for (int j = 0; j < NP; ++j) {
            combine_lines<T>(pr1, j, in, BE, tab, L, P, cr, dbuf + j * BE);
            crew_sync(cr);
            fft_line<T, -1, LC>(dbuf + j * BE, a.p, L, P, cr, twl);
        }
        __syncthreads();
    }

    if constexpr (PW == PW_UH) {
        // u = sum_p b0_p D_p (times V for V o N)   (Eq 94)
        for (int base = 0; base < E; base += kPwChunk * kThreads) {
            T b[kPwChunk][S], v[kPwChunk];
            long g[kPwChunk];
            int o[kPwChunk];
#pragma unroll
            for (int kk = 0; kk < kPwChunk; ++kk) {
                const int e = min(base + tid + kk * kThreads, E - 1);
                int w, i;
                tl.at(e, w, i, g[kk], o[kk]);
#pragma unroll
                for (int p = 0; p < S; ++p) b[kk][p] = m.b0[p * m.nn + g[kk]];
                v[kk] = m.vol ? m.vol[g[kk]] : T(1);
            }
#pragma unroll
            for (int kk = 0; kk < kPwChunk; ++kk) {
                if (base + tid + kk * kThreads < E) {
                    T acc = T(0);
#pragma unroll
                    for (int p = 0; p < S; ++p) {
                        cplx<T> c = dbuf[(p >> 1) * BE + o[kk]];
                        acc += b[kk][p] * ((p & 1) ? c.y : c.x);
                    }
                    reinterpret_cast<Tio*>(a.out)[g[kk]] = Tio(acc * v[kk]);
                }
            }
        }
        return;
    } else {
        if constexpr (PW == PW_K || PW == PW_KN) {
            // A^a = sum_q b^a_q D_q ; E_p = V sum_a b^a_p A^a   (Eq 90-91, Alg 2).
            // Interior nodes take the shared b^a and V (kernel argument) and
            // nodes outside the domain V = 0; only the others read the arrays.
            for (int base = 0; base < E; base += kPwChunk * kThreads) {
              T bb[kPwChunk][DIM][S], vv[kPwChunk];
              int oo[kPwChunk];
#pragma unroll
              for (int kk = 0; kk < kPwChunk; ++kk) {
                const int e = min(base + tid + kk * kThreads, E - 1);
                int w, i;
                long gi;
                tl.at(e, w, i, gi, oo[kk]);
                const uint8_t k = m.cls ? m.cls[gi] : uint8_t(2);
                // row sets wider than the interior constants have no classes
                // (cls NULL): every node reads the arrays
                if constexpr (DIM * S <= kMaxNodeConst) {
#pragma unroll
                    for (int al = 0; al < DIM; ++al)
#pragma unroll
                        for (int q = 0; q < S; ++q) bb[kk][al][q] = m.cint[al * S + q];
                    vv[kk] = k == 1 ? m.cint[DIM * S] : T(0);
                } else {
#pragma unroll
                    for (int al = 0; al < DIM; ++al)
#pragma unroll
                        for (int q = 0; q < S; ++q) bb[kk][al][q] = T(0);
                    vv[kk] = T(0);
                }
                if (k == 2) {
#pragma unroll
                    for (int al = 0; al < DIM; ++al)
#pragma unroll
                        for (int q = 0; q < S; ++q) bb[kk][al][q] = m.ba[(al * S + q) * m.nn + gi];
                    vv[kk] = m.vol[gi];
                }
              }
#pragma unroll
              for (int kk = 0; kk < kPwChunk; ++kk) {
                if (base + tid + kk * kThreads >= E) continue;
                const int o = oo[kk];
                T D[NP * 2];
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    cplx<T> c = dbuf[j * BE + o];
                    D[2 * j] = c.x;
                    D[2 * j + 1] = c.y;
                }
                T (&b)[DIM][S] = bb[kk];
                T A[DIM];
#pragma unroll
                for (int al = 0; al < DIM; ++al) {
                    T acc = T(0);
#pragma unroll
                    for (int q = 0; q < S; ++q) acc += b[al][q] * D[q];
                    A[al] = acc;
                }
                if constexpr (PW == PW_KN) {
                    // gradient nonlinearity N(A) = (1 + kappa |A|^2) A (Eq B.8, B.10)
                    T s2 = T(0);
#pragma unroll
                    for (int al = 0; al < DIM; ++al) s2 += A[al] * A[al];
                    const T f = T(1) + m.kappa * s2;
#pragma unroll
                    for (int al = 0; al < DIM; ++al) A[al] *= f;
                }
                const T v = vv[kk];
                T Ep[NP * 2];
#pragma unroll
                for (int p = 0; p < S; ++p) {
                    T acc = T(0);
#pragma unroll
                    for (int al = 0; al < DIM; ++al) acc += b[al][p] * A[al];
                    Ep[p] = v * acc;
                }
                if (S & 1) Ep[S] = T(0);
#pragma unroll
                for (int j = 0; j < NP; ++j) dbuf[j * BE + o] = cplx<T>{Ep[2 * j], Ep[2 * j + 1]};
              }
            }
        } else {
            // E_p = (V) b0_p r   (Eq 92, Alg 4)
            for (int base = 0; base < E; base += kPwChunk * kThreads) {
                T b[kPwChunk][S], x[kPwChunk];
                int o[kPwChunk];
#pragma unroll
                for (int kk = 0; kk < kPwChunk; ++kk) {
                    const int e = min(base + tid + kk * kThreads, E - 1);
                    int w, i;
                    long gi;
                    tl.at(e, w, i, gi, o[kk]);
                    x[kk] = T(reinterpret_cast<const Tio*>(msrc)[gi]) * (m.vol ? m.vol[gi] : T(1));
#pragma unroll
                    for (int p = 0; p < S; ++p) b[kk][p] = m.b0[p * m.nn + gi];
                }
#pragma unroll
                for (int kk = 0; kk < kPwChunk; ++kk) {
                    if (base + tid + kk * kThreads >= E) continue;
                    T Ep[NP * 2];
#pragma unroll
                    for (int p = 0; p < S; ++p) Ep[p] = b[kk][p] * x[kk];
                    if (S & 1) Ep[S] = T(0);
#pragma unroll
                    for (int j = 0; j < NP; ++j) dbuf[j * BE + o[kk]] = cplx<T>{Ep[2 * j], Ep[2 * j + 1]};
                }
            }
        }
        __syncthreads();
        for (int j = 0; j < NP; ++j) fft_line<T, +1, LC>(dbuf + j * BE, a.p, L, P, cr, twl);
        const int nbout = (m.nout2 + 1) / 2;
        const SepProg& pr2 = *m.pr2;
        double dacc = 0.0;
        for (int j = 0; j < nbout; ++j) {
            combine_lines<T>(pr2, j, dbuf, BE, tab, L, P, cr, work);
            crew_sync(cr);
            fft_line<T, -1, LC>(work, a.p, L, P, cr, twl);
            __syncthreads();
            dacc += store_tile<T, Tio, CONTIG, STM, LC>(a, tl, j, work, tid);
            __syncthreads();
        }
        if constexpr (STM == ST_REAL) {
            if (a.dot_part) {
                __shared__ double sh[kThreads / 64];
                double s = block_reduce(dacc, sh);
                if (tid == 0) a.dot_part[blockIdx.x] = s;
            }
        }
    }
}

// ------------------------------------------------------------ launchers

// tile width: the largest power of two W <= 16 with W*L <= max_tile that
// divides the line count (x axis) or the axis stride (other axes)
static AxisGeom sep_geom(const Ctx& c, int a, int max_tile, int wcap = 16)
{
    AxisGeom g;
    g.L = c.n[a];
    g.st = 1;
    for (int k = 0; k < a; ++k) g.st *= c.n[k];
    g.nlines = c.nn / g.L;
    g.contig = (g.st == 1);
    long div = g.contig ? g.nlines : g.st;
    int W = 16;
    while (W > 1 && (W > wcap || (long)W * g.L > max_tile || div % W != 0)) W >>= 1;
    g.W = W;
    g.wl = 0;
    while ((1 << g.wl) < W) ++g.wl;
    return g;
}

static size_t buf_bytes(const AxisGeom& g, size_t elem)
{
    return (size_t)g.W * (g.L + 1) * elem;
}

// Largest tile (elements per buffer, a power of two <= kMaxTile) whose nbuf
// buffers, row padding and kernel-spectrum table fit the LDS budget of a
// workgroup on axis a.
static int max_tile(const Ctx& c, int a, int nbuf, size_t elem)
{
    const size_t budget = (size_t)std::min(c.lds_budget, 65536) - 1024;
    const size_t tab = (size_t)(2 * c.degree + 2) * c.n[a] * elem;  // spectra + twiddles
    int t = kMaxTile;
    while (t > 64 && tab + (size_t)nbuf * (t + 16) * elem > budget) t >>= 1;
    return t;
}

template <typename T>
static void fill_common(const Ctx& c, int a, SepArgs<T>& s, int nbuf)
{
    // lines per workgroup: at most the setup-time choice of this precision
    s.g = sep_geom(c, a, max_tile(c, a, nbuf, sizeof(cplx<T>)), sizeof(T) == 8 ? c.sep_wcap[1] : c.sep_wcap[0]);
    s.p = c.plan[a];
    if constexpr (sizeof(T) == 8) {
        s.tw = c.tw64[a];
        s.tab = c.spec64[a];
    } else {
        s.tw = c.tw32[a];
        s.tab = c.spec32[a];
    }
    s.ne = 2 * c.degree + 1;
    s.fstride = c.nn;
}

size_t sep_lds_need(const Ctx& c, const SepPlan& sp, int elem_bytes)
{
    size_t worst = 0;
    const int np = (c.s + 1) / 2;
    for (int j = 0; j < sp.k; ++j) {
        const int a = c.axes[j];
        const int nin1 = (j == 0) ? 1 : sp.size[j - 1];
        int nbuf[2] = {(nin1 + 1) / 2 + 1, (sp.size[j] + 1) / 2 + 1};
        if (j == sp.k - 1) nbuf[1] = (nin1 + 1) / 2 + np + 1;  // middle pass
        for (int b = 0; b < 2; ++b) {
            AxisGeom g = sep_geom(c, a, max_tile(c, a, nbuf[b], elem_bytes));
            size_t need = (size_t)(2 * c.degree + 2) * g.L * elem_bytes + nbuf[b] * buf_bytes(g, elem_bytes);
            worst = std::max(worst, need);
        }
    }
    return worst;
}

static bool sep_log()
{
    static int on = -1;
    if (on < 0) {
        const char* e = getenv("FCRKPM_LOG");
        on = (e && *e >= '2') ? 1 : 0;
    }
    return on == 1;
}

template <typename T, typename Tio, bool CONTIG, int LDM, int STM>
static void go_pass(const SepArgs<T>& s, size_t sh, int nrhs, hipStream_t st)
{
    const dim3 grid((unsigned)(s.g.nlines / s.g.W), (unsigned)nrhs);
    if (s.g.L == 128)
        hipLaunchKernelGGL((k_sep_pass<T, Tio, CONTIG, LDM, STM, 128>), grid, dim3(kThreads), sh, st, s);
    else
        hipLaunchKernelGGL((k_sep_pass<T, Tio, CONTIG, LDM, STM, 0>), grid, dim3(kThreads), sh, st, s);
    if (sep_log()) {
        hipError_t e = hipPeekAtLastError();
        fprintf(stderr, "[fcrkpm] pass L=%d W=%d st=%ld contig=%d nin=%d nout=%d ld=%d st=%d lds=%zu T=%zu: %s\n",
                s.g.L, s.g.W, s.g.st, s.g.contig, s.nin, s.nout, LDM, STM, sh, sizeof(T),
                hipGetErrorString(e));
    }
}

template <typename T, typename Tio>
void launch_sep_pass(const Ctx& c, int a, const SepProg& pr, const SepProg* dpr, int ldm,
                     const void* in, const uint8_t* mask_in, int stm, void* out,
                     const uint8_t* mask_out, double* dot_part, const void* dot_with,
                     hipStream_t st, const RhsBatch& rb)
{
    SepArgs<T> s;
    s.in_rb = rb.in_bytes;
    s.out_rb = rb.out_bytes;
    const int nbin = (pr.nin + 1) / 2;
    fill_common<T>(c, a, s, nbin + 1);
    s.in = in;
    s.mask_in = mask_in;
    s.out = out;
    s.mask_out = mask_out;
    s.pr = dpr;
    s.nin = pr.nin;
    s.nout = pr.nout;
    s.dot_part = dot_part;
    s.dot_with = dot_with;
    const size_t sh = (size_t)(s.ne + 1) * s.g.L * sizeof(cplx<T>) + (nbin + 1) * buf_bytes(s.g, sizeof(cplx<T>));
#define FC_PASS(CT, LD, STO) go_pass<T, Tio, CT, LD, STO>(s, sh, rb.n, st)
    const bool ct = s.g.contig;
    if (ldm == LD_PAIRS && stm == ST_PAIRS) { if (ct) FC_PASS(true, LD_PAIRS, ST_PAIRS); else FC_PASS(false, LD_PAIRS, ST_PAIRS); }
    else if (ldm == LD_REAL && stm == ST_PAIRS) { if (ct) FC_PASS(true, LD_REAL, ST_PAIRS); else FC_PASS(false, LD_REAL, ST_PAIRS); }
    else if (ldm == LD_CHI && stm == ST_PAIRS) { if (ct) FC_PASS(true, LD_CHI, ST_PAIRS); else FC_PASS(false, LD_CHI, ST_PAIRS); }
    else if (ldm == LD_PAIRS && stm == ST_REAL) { if (ct) FC_PASS(true, LD_PAIRS, ST_REAL); else FC_PASS(false, LD_PAIRS, ST_REAL); }
#undef FC_PASS
}

template <typename T, typename Tio, bool CONTIG, int LDM, int STM, int S, int DIM, int PW>
static void go_mid(const MidArgs<T>& m, size_t sh, int nrhs, hipStream_t st)
{
    const dim3 grid((unsigned)(m.s.g.nlines / m.s.g.W), (unsigned)nrhs);
    // the 128-point lines of the 3D workloads (bases of 4 and 10 monomials)
    // get the compile-time plan
    if constexpr ((S == 4 || S == 10) && !CONTIG) {
        if (m.s.g.L == 128) {
            hipLaunchKernelGGL((k_sep_mid<T, Tio, CONTIG, LDM, STM, S, DIM, PW, 128>), grid,
                               dim3(kThreads), sh, st, m);
            return;
        }
    }
    hipLaunchKernelGGL((k_sep_mid<T, Tio, CONTIG, LDM, STM, S, DIM, PW, 0>), grid, dim3(kThreads),
                       sh, st, m);
    if (sep_log()) {
        hipError_t e = hipPeekAtLastError();
        fprintf(stderr, "[fcrkpm] mid L=%d W=%d st=%ld pw=%d nin=%d nout2=%d lds=%zu T=%zu: %s\n",
                m.s.g.L, m.s.g.W, m.s.g.st, PW, m.s.nin, m.nout2, sh, sizeof(T),
                hipGetErrorString(e));
    }
}

// DIM is the number of coefficient rows of the K-type pointwise stage; KONLY
// instantiates that stage alone (row counts other than the dimension: the
// mass and shifted products of time-dependent problems)
template <typename T, typename Tio, int S, int DIM, bool KONLY = false>
static void mid_dispatch(const MidArgs<T>& m, int ldm, int stm, int pw, size_t sh, int nrhs,
                         hipStream_t st)
{
    const bool ct = m.s.g.contig;
#define FC_MID(CT, LD, STO, P) go_mid<T, Tio, CT, LD, STO, S, DIM, P>(m, sh, nrhs, st)
    if constexpr (KONLY) {
        if (pw != PW_K) raise_unsupported("internal: pointwise mode without its instantiation");
        if (ldm == LD_REAL && stm == ST_REAL) { if (ct) FC_MID(true, LD_REAL, ST_REAL, PW_K); else FC_MID(false, LD_REAL, ST_REAL, PW_K); }
        else { if (ct) FC_MID(true, LD_PAIRS, ST_PAIRS, PW_K); else FC_MID(false, LD_PAIRS, ST_PAIRS, PW_K); }
    } else if (pw == PW_KN) {
        if constexpr (std::is_same<T, double>::value && std::is_same<Tio, double>::value) {
            if (ldm == LD_REAL && stm == ST_REAL) { if (ct) FC_MID(true, LD_REAL, ST_REAL, PW_KN); else FC_MID(false, LD_REAL, ST_REAL, PW_KN); }
            else { if (ct) FC_MID(true, LD_PAIRS, ST_PAIRS, PW_KN); else FC_MID(false, LD_PAIRS, ST_PAIRS, PW_KN); }
        } else {
            raise_unsupported("the gradient nonlinearity runs in FP64 only");
        }
    } else if (pw == PW_K) {
        if (ldm == LD_REAL && stm == ST_REAL) { if (ct) FC_MID(true, LD_REAL, ST_REAL, PW_K); else FC_MID(false, LD_REAL, ST_REAL, PW_K); }
        else { if (ct) FC_MID(true, LD_PAIRS, ST_PAIRS, PW_K); else FC_MID(false, LD_PAIRS, ST_PAIRS, PW_K); }
    } else if (pw == PW_UH) {
        if (ldm == LD_REAL) { if (ct) FC_MID(true, LD_REAL, ST_REAL, PW_UH); else FC_MID(false, LD_REAL, ST_REAL, PW_UH); }
        else { if (ct) FC_MID(true, LD_PAIRS, ST_REAL, PW_UH); else FC_MID(false, LD_PAIRS, ST_REAL, PW_UH); }
    } else {
        if (stm == ST_REAL) { if (ct) FC_MID(true, LD_PAIRS, ST_REAL, PW_LOAD); else FC_MID(false, LD_PAIRS, ST_REAL, PW_LOAD); }
        else { if (ct) FC_MID(true, LD_PAIRS, ST_PAIRS, PW_LOAD); else FC_MID(false, LD_PAIRS, ST_PAIRS, PW_LOAD); }
    }
#undef FC_MID
}

template <typename T, typename Tio>
void launch_sep_mid(const Ctx& c, int a, const SepProg& pr1, const SepProg* dpr1,
                    const SepProg& pr2, const SepProg* dpr2, int pw, int ldm,
                    const void* in, const uint8_t* mask_in, int stm, void* out,
                    const uint8_t* mask_out, const void* src, const T* b0, const T* ba,
                    const T* vol, double* dot_part, const void* dot_with, hipStream_t st,
                    const RhsBatch& rb)
{
    MidArgs<T> m;
    m.s.in_rb = rb.in_bytes;
    m.s.out_rb = rb.out_bytes;
    m.src_rb = rb.src_bytes;
    const int np = (c.s + 1) / 2;
    const int nbin = (pw == PW_LOAD) ? 0 : (pr1.nin + 1) / 2;
    const int nbuf = nbin + np + (pw == PW_UH ? 0 : 1);
    fill_common<T>(c, a, m.s, nbuf);
    m.s.in = in;
    m.s.mask_in = mask_in;
    m.s.out = out;
    m.s.mask_out = mask_out;
    m.s.pr = dpr1;
    m.s.nin = pr1.nin;
    m.s.nout = pr1.nout;
    m.s.dot_part = dot_part;
    m.s.dot_with = dot_with;
    m.pr2 = dpr2;
    m.nout2 = pr2.nout;
    m.b0 = b0;
    m.ba = ba;
    m.vol = vol;
    m.cls = c.cls;
    m.kappa = (T)c.pw_kappa;
    for (int q = 0; q <= kMaxNodeConst; ++q) {
        if constexpr (std::is_same<T, double>::value) m.cint[q] = c.cint64[q];
        else m.cint[q] = c.cint32[q];
    }
    m.src = src;
    m.nn = c.nn;
    const size_t sh = (size_t)(m.s.ne + 1) * m.s.g.L * sizeof(cplx<T>) + nbuf * buf_bytes(m.s.g, sizeof(cplx<T>));
    const int rows = (pw == PW_K || pw == PW_KN) ? c.krows : c.dim;
    if (rows == c.dim) {
        if (c.s == 2 && c.dim == 1) mid_dispatch<T, Tio, 2, 1>(m, ldm, stm, pw, sh, rb.n, st);
        else if (c.s == 3 && c.dim == 1) mid_dispatch<T, Tio, 3, 1>(m, ldm, stm, pw, sh, rb.n, st);
        else if (c.s == 3 && c.dim == 2) mid_dispatch<T, Tio, 3, 2>(m, ldm, stm, pw, sh, rb.n, st);
        else if (c.s == 6 && c.dim == 2) mid_dispatch<T, Tio, 6, 2>(m, ldm, stm, pw, sh, rb.n, st);
        else if (c.s == 4 && c.dim == 3) mid_dispatch<T, Tio, 4, 3>(m, ldm, stm, pw, sh, rb.n, st);
        else if (c.s == 10 && c.dim == 3) mid_dispatch<T, Tio, 10, 3>(m, ldm, stm, pw, sh, rb.n, st);
        else if (c.s == 4 && c.dim == 1) mid_dispatch<T, Tio, 4, 1>(m, ldm, stm, pw, sh, rb.n, st);   // cubic, 1D
        else if (c.s == 10 && c.dim == 2) mid_dispatch<T, Tio, 10, 2>(m, ldm, stm, pw, sh, rb.n, st);  // cubic, 2D
        else raise_unsupported("basis size and dimension without a middle pass");
        return;
    }
    // the consistent mass (one row) and c_m M + c_k K (dim + 1 rows)
    if (c.s == 2 && rows == 2) mid_dispatch<T, Tio, 2, 2, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 3 && rows == 1) mid_dispatch<T, Tio, 3, 1, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 3 && rows == 2) mid_dispatch<T, Tio, 3, 2, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 3 && rows == 3) mid_dispatch<T, Tio, 3, 3, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 6 && rows == 1) mid_dispatch<T, Tio, 6, 1, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 6 && rows == 3) mid_dispatch<T, Tio, 6, 3, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 4 && rows == 1) mid_dispatch<T, Tio, 4, 1, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 4 && rows == 4) mid_dispatch<T, Tio, 4, 4, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 10 && rows == 1) mid_dispatch<T, Tio, 10, 1, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 10 && rows == 4) mid_dispatch<T, Tio, 10, 4, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 4 && rows == 2) mid_dispatch<T, Tio, 4, 2, true>(m, ldm, stm, pw, sh, rb.n, st);
    else if (c.s == 10 && rows == 3) mid_dispatch<T, Tio, 10, 3, true>(m, ldm, stm, pw, sh, rb.n, st);
    else raise_unsupported("coefficient rows without a middle pass");
}

template void launch_sep_pass<double, double>(const Ctx&, int, const SepProg&, const SepProg*, int, const void*,
                                              const uint8_t*, int, void*, const uint8_t*, double*,
                                              const void*, hipStream_t, const RhsBatch&);
template void launch_sep_pass<float, float>(const Ctx&, int, const SepProg&, const SepProg*, int, const void*,
                                            const uint8_t*, int, void*, const uint8_t*, double*,
                                            const void*, hipStream_t, const RhsBatch&);
template void launch_sep_pass<float, double>(const Ctx&, int, const SepProg&, const SepProg*, int, const void*,
                                             const uint8_t*, int, void*, const uint8_t*, double*,
                                             const void*, hipStream_t, const RhsBatch&);
template void launch_sep_mid<float, double>(const Ctx&, int, const SepProg&, const SepProg*, const SepProg&, const SepProg*, int,
                                            int, const void*, const uint8_t*, int, void*,
                                            const uint8_t*, const void*, const float*, const float*,
                                            const float*, double*, const void*, hipStream_t, const RhsBatch&);
template void launch_sep_mid<double, double>(const Ctx&, int, const SepProg&, const SepProg*, const SepProg&, const SepProg*, int,
                                             int, const void*, const uint8_t*, int, void*,
                                             const uint8_t*, const void*, const double*,
                                             const double*, const double*, double*, const void*,
                                             hipStream_t, const RhsBatch&);
template void launch_sep_mid<float, float>(const Ctx&, int, const SepProg&, const SepProg*, const SepProg&, const SepProg*, int,
                                           int, const void*, const uint8_t*, int, void*,
                                           const uint8_t*, const void*, const float*, const float*,
                                           const float*, double*, const void*, hipStream_t, const RhsBatch&);

}  // namespace fcrkpm
