// kernels.hip -- gfx950 setup and vector kernels of the FC-RKPM Poisson path.
//
//  * k_moment_solve: per-node FP64 Cholesky of the s x s moment matrix and the
//                   rows of M^-1 that give b^0 and b^a (Alg 1, Eq 83-85).
//  * CG vectors   : fused axpy + dot with deterministic two-stage reductions.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fcrkpm_impl.hpp"

namespace fcrkpm {

static unsigned ew_blocks(long n)
{
    long b = (n + 255) / 256;
    if (b > 65535L * 8) b = 65535L * 8;
    return (unsigned)(b < 1 ? 1 : b);
}

#define FCRKPM_DISPATCH_S(S_, DIM_, ...)                                                     \
    if (c.s == 2 && c.dim == 1) { constexpr int S_ = 2, DIM_ = 1; (void)DIM_; __VA_ARGS__; }      \
    else if (c.s == 3 && c.dim == 1) { constexpr int S_ = 3, DIM_ = 1; (void)DIM_; __VA_ARGS__; } \
    else if (c.s == 3 && c.dim == 2) { constexpr int S_ = 3, DIM_ = 2; (void)DIM_; __VA_ARGS__; } \
    else if (c.s == 6 && c.dim == 2) { constexpr int S_ = 6, DIM_ = 2; (void)DIM_; __VA_ARGS__; } \
    else if (c.s == 4 && c.dim == 3) { constexpr int S_ = 4, DIM_ = 3; (void)DIM_; __VA_ARGS__; } \
    else if (c.s == 10 && c.dim == 3) { constexpr int S_ = 10, DIM_ = 3; (void)DIM_; __VA_ARGS__; } \
    else if (c.s == 4 && c.dim == 1) { constexpr int S_ = 4, DIM_ = 1; (void)DIM_; __VA_ARGS__; }   \
    else if (c.s == 10 && c.dim == 2) { constexpr int S_ = 10, DIM_ = 2; (void)DIM_; __VA_ARGS__; }

// ============================================================ setup kernels

__global__ void k_free_mask(const uint8_t* __restrict__ chi, const uint8_t* __restrict__ dir,
                            uint8_t* __restrict__ freem, int* bad, long nn)
{
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < nn;
         I += (long)gridDim.x * blockDim.x) {
        uint8_t c = chi[I] ? 1 : 0;
        uint8_t d = (dir && dir[I]) ? 1 : 0;
        if (d && !c) atomicMin(bad, (int)I);
        freem[I] = (c && !d) ? 1 : 0;
    }
}

void launch_free_mask(const uint8_t* chi, const uint8_t* dir, uint8_t* freem, int* bad, long nn,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_free_mask, dim3(ew_blocks(nn)), dim3(256), 0, st, chi, dir, freem, bad,
                       nn);
}

// occ[off_a + i] = 1 if some domain node has coordinate i on axis a
__global__ void k_axis_extent(const uint8_t* __restrict__ chi, int n0, int n1, int n2, int* occ,
                              long nn)
{
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < nn;
         I += (long)gridDim.x * blockDim.x) {
        if (!chi[I]) continue;
        int i0 = (int)(I % n0);
        long r = I / n0;
        int i1 = (int)(r % n1);
        int i2 = (int)(r / n1);
        occ[i0] = 1;
        occ[n0 + i1] = 1;
        occ[n0 + n1 + i2] = 1;
    }
}

void launch_axis_extent(const Ctx& c, const uint8_t* chi, int* occ, hipStream_t st)
{
    hipLaunchKernelGGL(k_axis_extent, dim3(ew_blocks(c.nn)), dim3(256), 0, st, chi, c.n[0],
                       c.n[1], c.n[2], occ, c.nn);
}

// Node classes for the pointwise stage of the FP32 K product: 0 outside the
// domain, 1 a node whose whole support neighbourhood (periodic, as the
// convolutions see it) lies in the domain and whose b^a and V equal the
// reference interior values to FP32 precision, 2 any other domain node.
__device__ __forceinline__ bool full_support(const uint8_t* __restrict__ chi, long I, int n0, int n1,
                                             int n2, int m0, int m1, int m2)
{
    const int i0 = (int)(I % n0);
    const long r = I / n0;
    const int i1 = (int)(r % n1), i2 = (int)(r / n1);
    for (int o2 = -m2; o2 <= m2; ++o2) {
        const int j2 = (i2 + o2 + n2) % n2;
        for (int o1 = -m1; o1 <= m1; ++o1) {
            const int j1 = (i1 + o1 + n1) % n1;
            const long row = ((long)j2 * n1 + j1) * n0;
            for (int o0 = -m0; o0 <= m0; ++o0)
                if (!chi[row + (i0 + o0 + n0) % n0]) return false;
        }
    }
    return true;
}

__global__ void k_first_interior(const uint8_t* __restrict__ chi, int n0, int n1, int n2, int m0,
                                 int m1, int m2, long nn, int* ref)
{
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < nn;
         I += (long)gridDim.x * blockDim.x)
        if (chi[I] && full_support(chi, I, n0, n1, n2, m0, m1, m2)) atomicMin(ref, (int)I);
}

void launch_first_interior(const Ctx& c, int* ref, hipStream_t st)
{
    hipLaunchKernelGGL(k_first_interior, dim3(ew_blocks(c.nn)), dim3(256), 0, st, c.chi, c.n[0],
                       c.n[1], c.n[2], c.m[0], c.m[1], c.m[2], c.nn, ref);
}

__global__ void k_node_class(const uint8_t* __restrict__ chi, const double* __restrict__ ba,
                             const double* __restrict__ vol, int nb, NodeConst ref, int n0, int n1,
                             int n2, int m0, int m1, int m2, long nn, uint8_t* __restrict__ cls)
{
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < nn;
         I += (long)gridDim.x * blockDim.x) {
        uint8_t k = 0;
        if (chi[I]) {
            bool same = ref.bmax >= 0.0 && vol[I] == ref.v && full_support(chi, I, n0, n1, n2, m0, m1, m2);
            for (int q = 0; same && q < nb; ++q)
                same = fabs(ba[(long)q * nn + I] - ref.b[q]) <= 1e-12 * ref.bmax;
            k = same ? 1 : 2;
        }
        cls[I] = k;
    }
}

void launch_node_class(const Ctx& c, const NodeConst& ref, uint8_t* cls, hipStream_t st)
{
    hipLaunchKernelGGL(k_node_class, dim3(ew_blocks(c.nn)), dim3(256), 0, st, c.chi, c.ba_64,
                       c.vol64, c.krows * c.s, ref, c.n[0], c.n[1], c.n[2], c.m[0], c.m[1], c.m[2],
                       c.nn, cls);
}

__global__ void k_vol(const uint8_t* __restrict__ chi, const double* __restrict__ vin, double hv,
                      double* __restrict__ v64, float* __restrict__ v32, long nn)
{
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < nn;
         I += (long)gridDim.x * blockDim.x) {
        double v = vin ? vin[I] : (chi[I] ? hv : 0.0);
        v64[I] = v;
        v32[I] = (float)v;
    }
}

void launch_vol(const uint8_t* chi, const double* vol_in, double hv, double* vol64, float* vol32,
                long nn, hipStream_t st)
{
    hipLaunchKernelGGL(k_vol, dim3(ew_blocks(nn)), dim3(256), 0, st, chi, vol_in, hv, vol64, vol32,
                       nn);
}

__global__ void k_mask_to_double(const uint8_t* __restrict__ m, double* __restrict__ out, long nn)
{
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < nn;
         I += (long)gridDim.x * blockDim.x)
        out[I] = m[I] ? 1.0 : 0.0;
}

void launch_mask_to_double(const uint8_t* m, double* out, long nn, hipStream_t st)
{
    hipLaunchKernelGGL(k_mask_to_double, dim3(ew_blocks(nn)), dim3(256), 0, st, m, out, nn);
}

__global__ void k_check_finite(const double* __restrict__ x, long nn, int* flag)
{
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < nn;
         I += (long)gridDim.x * blockDim.x)
        if (!isfinite(x[I])) atomicOr(flag, 1);
}

void launch_check_finite(const double* x, long nn, int* flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_finite, dim3(ew_blocks(nn)), dim3(256), 0, st, x, nn, flag);
}

// Per-node moment matrix from the monomial convolutions G (pairs), Cholesky,
// b^0 = M^-1 e_1, b^a = -M^-1 e_{1+a} / h_a; zero where chi = 0 (Eq 48 gives
// M = I there and every use is masked).  Pivot <= 1e-13 trace -> singular.
struct MomentArgs {
    int8_t pq2m[kMaxS * kMaxS];
    double invh[3];
};

template <int S, int DIM>
__global__ __launch_bounds__(64) void k_moment_solve(const cplx<double>* __restrict__ G, const uint8_t* __restrict__ chi,
                               long nn, MomentArgs ma, double* __restrict__ b0,
                               double* __restrict__ ba, float* __restrict__ b0f,
                               float* __restrict__ baf, int* bad)
{
    for (long I = blockIdx.x * (long)blockDim.x + threadIdx.x; I < nn;
         I += (long)gridDim.x * blockDim.x) {
        double Lm[S][S];
        bool ok = chi[I] != 0;
        if (ok) {
            double tr = 0.0;
#pragma unroll
            for (int p = 0; p < S; ++p)
#pragma unroll
                for (int q = 0; q <= p; ++q) {
                    int m = ma.pq2m[p * S + q];
                    cplx<double> g = G[(long)(m >> 1) * nn + I];
                    Lm[p][q] = (m & 1) ? g.y : g.x;
                }
#pragma unroll
            for (int p = 0; p < S; ++p) tr += Lm[p][p];
            const double tol = 1e-13 * tr;
#pragma unroll
            for (int j = 0; j < S; ++j) {
                double d = Lm[j][j];
#pragma unroll
                for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
                if (!(d > tol)) ok = false;
                d = sqrt(d > 0.0 ? d : 1.0);
                Lm[j][j] = d;
                const double id = 1.0 / d;
#pragma unroll
                for (int i = j + 1; i < S; ++i) {
                    double v = Lm[i][j];
#pragma unroll
                    for (int k = 0; k < j; ++k) v -= Lm[i][k] * Lm[j][k];
                    Lm[i][j] = v * id;
                }
            }
            if (!ok) atomicMin(bad, (int)I);
        }
#pragma unroll
        for (int col = 0; col <= DIM; ++col) {
            double y[S];
            if (ok) {
                double z[S];
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    double v = (i == col) ? 1.0 : 0.0;
#pragma unroll
                    for (int k = 0; k < i; ++k) v -= Lm[i][k] * z[k];
                    z[i] = v / Lm[i][i];
                }
#pragma unroll
                for (int i = S - 1; i >= 0; --i) {
                    double v = z[i];
#pragma unroll
                    for (int k = i + 1; k < S; ++k) v -= Lm[k][i] * y[k];
                    y[i] = v / Lm[i][i];
                }
            } else {
#pragma unroll
                for (int i = 0; i < S; ++i) y[i] = 0.0;
            }
            if (col == 0) {
#pragma unroll
                for (int p = 0; p < S; ++p) {
                    b0[p * nn + I] = y[p];
                    b0f[p * nn + I] = (float)y[p];
                }
            } else {
                const double sc = -ma.invh[col - 1];
#pragma unroll
                for (int p = 0; p < S; ++p) {
                    double v = y[p] * sc;
                    ba[((col - 1) * S + p) * nn + I] = v;
                    baf[((col - 1) * S + p) * nn + I] = (float)v;
                }
            }
        }
    }
}

static int mono_index(const Ctx& c, int e0, int e1, int e2)
{
    for (int m = 0; m < c.nmono2; ++m)
        if (c.ex2[m][0] == e0 && c.ex2[m][1] == e1 && c.ex2[m][2] == e2) return m;
    return -1;
}

void launch_moment_solve(const Ctx& c, const cplx<double>* G, int* bad, hipStream_t st)
{
    MomentArgs ma;
    for (int p = 0; p < c.s; ++p)
        for (int q = 0; q < c.s; ++q)
            ma.pq2m[p * c.s + q] = (int8_t)mono_index(c, c.ex[p][0] + c.ex[q][0],
                                                      c.ex[p][1] + c.ex[q][1],
                                                      c.ex[p][2] + c.ex[q][2]);
    for (int a = 0; a < 3; ++a) ma.invh[a] = 1.0 / c.h[a];
    // one node per thread; the register-resident factor is large for s = 10,
    // so workgroups are one wave
    long b = (c.nn + 63) / 64;
    unsigned blocks = (unsigned)std::min(b, 65535L * 32);
    FCRKPM_DISPATCH_S(S, DIM, hipLaunchKernelGGL((k_moment_solve<S, DIM>), dim3(blocks),
                                                   dim3(64), 0, st, G, c.chi, c.nn, ma, c.b0_64,
                                                   c.ba_64, c.b0_32, c.ba_32, bad));
}

// ============================================================ CG vector kernels

__device__ __forceinline__ double block_sum(double v, double* sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
    return r;
}

// Batched reductions: right-hand side j = blockIdx.y owns vectors at offset
// j*n, nb partials at j*kRedBlocks and kScal scalars at j*kScal.  The number
// of partials nb depends on n only, and every block sums them in the same
// fixed order, so results are bitwise reproducible.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nb, double* sh)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
    return block_sum(v, sh);
}

// sum_partials in two steps for blocks of kRedThreads threads over a
// right-hand side's kRedBlocks partial slots: load (all slots, without
// branches, so that loads issued after them do not delay the sum), then sum
// (the first nb slots, in the order of sum_partials)
struct Partials {
    double v[kRedBlocks / kRedThreads];
    __device__ __forceinline__ void load(const double* __restrict__ part)
    {
#pragma unroll
        for (int k = 0; k < kRedBlocks / kRedThreads; ++k) v[k] = part[threadIdx.x + k * kRedThreads];
    }
    __device__ __forceinline__ double sum(int nb, double* sh) const
    {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kRedBlocks / kRedThreads; ++k)
            if ((int)threadIdx.x + k * kRedThreads < nb) s += v[k];
        return block_sum(s, sh);
    }
};

// chunks of four a CG update thread loads ahead of its block's reduction
constexpr int kPre = 2;

int red_blocks(long n)
{
    const long per = (long)kRedThreads * 4;
    return (int)std::max(1L, std::min((long)kRedBlocks, (n + per - 1) / per));
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_dot_partial(const T* __restrict__ a,
                                                             const T* __restrict__ b, long n,
                                                             double* __restrict__ part,
                                                             const int* __restrict__ act)
{
    __shared__ double sh[16];
    const int j = blockIdx.y;
    if (act && !act[j]) return;
    a += j * n;
    b += j * n;
    double acc = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        acc += (double)a[i] * (double)b[i];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(long)j * kRedBlocks + blockIdx.x] = s;
}

template <typename T>
void launch_dot_partial(const T* a, const T* b, long n, int nrhs, double* part, const int* act,
                        hipStream_t st)
{
    hipLaunchKernelGGL((k_dot_partial<T>), dim3(red_blocks(n), nrhs), dim3(kRedThreads), 0, st,
                       a, b, n, part, act);
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_to(const double* __restrict__ part, int nb,
                                                           double* dst)
{
    __shared__ double sh[16];
    const int j = blockIdx.y;
    double s = sum_partials(part + (long)j * kRedBlocks, nb, sh);
    if (threadIdx.x == 0) dst[j * kScal] = s;
}

void launch_reduce_to(const double* part, long n, int nrhs, double* dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_to, dim3(1, nrhs), dim3(kRedThreads), 0, st, part, red_blocks(n),
                       dst);
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_wide(const double* __restrict__ part, int nb,
                                                             long stride, double* dst)
{
    __shared__ double sh[16];
    const int j = blockIdx.y;
    double s = sum_partials(part + (long)j * stride, nb, sh);
    if (threadIdx.x == 0) dst[(long)j * kRedBlocks] = s;
}

void launch_reduce_wide(const double* part, int nb, long stride, int nrhs, double* dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_wide, dim3(1, nrhs), dim3(kRedThreads), 0, st, part, nb, stride, dst);
}

// scalars of one right-hand side: [0], [1] = r.r (double-buffered by
// parity), [3] = breakdown flag.  Right-hand sides with act[j] == 0 are
// frozen: x, r, p and their scalars stay as they are.
// Four consecutive elements per thread and step: FP32 vectors move as float4
// when the field length allows it (n % 4 == 0, fields then stay 16-byte
// aligned), otherwise one element at a time.
template <typename T>
struct Vec4 {
    T v[4];
};
template <typename T>
__device__ __forceinline__ Vec4<T> ld4(const T* p)
{
    Vec4<T> o;
    if constexpr (sizeof(T) == 4) {
        const float4 f = *reinterpret_cast<const float4*>(p);
        o.v[0] = f.x;
        o.v[1] = f.y;
        o.v[2] = f.z;
        o.v[3] = f.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        o.v[0] = a.x;
        o.v[1] = a.y;
        o.v[2] = b.x;
        o.v[3] = b.y;
    }
    return o;
}
template <typename T>
__device__ __forceinline__ void st4(T* p, const Vec4<T>& o)
{
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = float4{o.v[0], o.v[1], o.v[2], o.v[3]};
    } else {
        *reinterpret_cast<double2*>(p) = double2{o.v[0], o.v[1]};
        *reinterpret_cast<double2*>(p + 2) = double2{o.v[2], o.v[3]};
    }
}

// npq: the number of p.q partials of each right-hand side (written by
// k_dot_partial, or by the last pass of the K product)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_cg_xr(T* __restrict__ x, T* __restrict__ r,
                                                       const T* __restrict__ p,
                                                       const T* __restrict__ q, long n,
                                                       const double* __restrict__ pq_part, int npq,
                                                       double* scal, int parity,
                                                       double* __restrict__ rr_part,
                                                       const int* __restrict__ act)
{
    __shared__ double sh[16];
    const int j = blockIdx.y;
    if (!act[j]) return;
    const long off = j * n;
    x += off;
    r += off;
    p += off;
    q += off;
    scal += j * kScal;
    const long stride = (long)gridDim.x * blockDim.x;
    const long first = blockIdx.x * (long)blockDim.x + threadIdx.x;
    // the partials of p.q, then the thread's first kPre chunks are loaded
    // before the reduction, so the chunks' latency overlaps it
    Partials pp;
    pp.load(pq_part + (long)j * kRedBlocks);
    Vec4<T> xs[kPre], rs[kPre], ps[kPre], qs[kPre];
    if (n % 4 == 0) {
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const long i = 4 * (first + u * stride);
            if (i < n) {
                xs[u] = ld4(x + i);
                rs[u] = ld4(r + i);
                ps[u] = ld4(p + i);
                qs[u] = ld4(q + i);
            }
        }
    }
    const double pq = pp.sum(npq, sh);
    const double rr = scal[parity];
    const bool good = pq > 0.0 && rr > 0.0;
    const T alpha = good ? T(rr / pq) : T(0);
    if (!good && blockIdx.x == 0 && threadIdx.x == 0 && rr > 0.0) scal[3] = 1.0;
    double acc = 0.0;
    if (n % 4 == 0) {
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const long i = 4 * (first + u * stride);
            if (i < n) {
                Vec4<T> xv = xs[u], rv = rs[u];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xv.v[e] = xv.v[e] + alpha * ps[u].v[e];
                    rv.v[e] = rv.v[e] - alpha * qs[u].v[e];
                    acc += (double)rv.v[e] * (double)rv.v[e];
                }
                st4(x + i, xv);
                st4(r + i, rv);
            }
        }
        for (long i = 4 * (first + kPre * stride); i < n; i += 4 * stride) {
            Vec4<T> xv = ld4(x + i), rv = ld4(r + i);
            const Vec4<T> pv = ld4(p + i), qv = ld4(q + i);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv.v[u] = xv.v[u] + alpha * pv.v[u];
                rv.v[u] = rv.v[u] - alpha * qv.v[u];
                acc += (double)rv.v[u] * (double)rv.v[u];
            }
            st4(x + i, xv);
            st4(r + i, rv);
        }
    } else {
        for (long i = first; i < n; i += stride) {
            T xi = x[i] + alpha * p[i];
            T ri = r[i] - alpha * q[i];
            x[i] = xi;
            r[i] = ri;
            acc += (double)ri * (double)ri;
        }
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) rr_part[(long)j * kRedBlocks + blockIdx.x] = s;
}

template <typename T>
void launch_cg_xr(T* x, T* r, const T* p, const T* q, long n, int nrhs, const double* pq_part,
                  int npq, double* scal, int parity, double* rr_part, const int* act,
                  hipStream_t st)
{
    hipLaunchKernelGGL((k_cg_xr<T>), dim3(red_blocks(n), nrhs), dim3(kRedThreads), 0, st, x, r, p,
                       q, n, pq_part, npq, scal, parity, rr_part, act);
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_cg_p(T* __restrict__ p, const T* __restrict__ r,
                                                      long n, const double* __restrict__ rr_part,
                                                      double* scal, int parity,
                                                      const int* __restrict__ act)
{
    __shared__ double sh[16];
    const int j = blockIdx.y;
    if (!act[j]) return;
    p += j * n;
    r += j * n;
    scal += j * kScal;
    const long stride = (long)gridDim.x * blockDim.x;
    const long first = blockIdx.x * (long)blockDim.x + threadIdx.x;
    Partials pp;
    pp.load(rr_part + (long)j * kRedBlocks);
    Vec4<T> rs[kPre], ps[kPre];
    if (n % 4 == 0) {
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const long i = 4 * (first + u * stride);
            if (i < n) {
                rs[u] = ld4(r + i);
                ps[u] = ld4(p + i);
            }
        }
    }
    const double rr_new = pp.sum(gridDim.x, sh);
    const double rr_old = scal[parity];
    const T beta = rr_old > 0.0 ? T(rr_new / rr_old) : T(0);
    if (n % 4 == 0) {
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const long i = 4 * (first + u * stride);
            if (i < n) {
                Vec4<T> pv = ps[u];
#pragma unroll
                for (int e = 0; e < 4; ++e) pv.v[e] = rs[u].v[e] + beta * pv.v[e];
                st4(p + i, pv);
            }
        }
        for (long i = 4 * (first + kPre * stride); i < n; i += 4 * stride) {
            const Vec4<T> rv = ld4(r + i);
            Vec4<T> pv = ld4(p + i);
#pragma unroll
            for (int u = 0; u < 4; ++u) pv.v[u] = rv.v[u] + beta * pv.v[u];
            st4(p + i, pv);
        }
    } else {
        for (long i = first; i < n; i += stride) p[i] = r[i] + beta * p[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[1 - parity] = rr_new;
}

template <typename T>
void launch_cg_p(T* p, const T* r, long n, int nrhs, const double* rr_part, double* scal,
                 int parity, const int* act, hipStream_t st)
{
    hipLaunchKernelGGL((k_cg_p<T>), dim3(red_blocks(n), nrhs), dim3(kRedThreads), 0, st, p, r, n,
                       rr_part, scal, parity, act);
}

template void launch_dot_partial<double>(const double*, const double*, long, int, double*,
                                         const int*, hipStream_t);
template void launch_dot_partial<float>(const float*, const float*, long, int, double*,
                                        const int*, hipStream_t);
template void launch_cg_xr<double>(double*, double*, const double*, const double*, long, int,
                                   const double*, int, double*, int, double*, const int*,
                                   hipStream_t);
template void launch_cg_xr<float>(float*, float*, const float*, const float*, long, int,
                                  const double*, int, double*, int, double*, const int*,
                                  hipStream_t);
template void launch_cg_p<double>(double*, const double*, long, int, const double*, double*, int,
                                  const int*, hipStream_t);
template void launch_cg_p<float>(float*, const float*, long, int, const double*, double*, int,
                                 const int*, hipStream_t);

// scal[j*kScal + idx] = v for every right-hand side
__global__ void k_set_scalar(double* scal, int idx, double v, int nrhs)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nrhs) scal[j * kScal + idx] = v;
}

void launch_set_scalar(double* scal, int idx, double v, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_scalar, dim3((nrhs + 63) / 64), dim3(64), 0, st, scal, idx, v, nrhs);
}

__global__ void k_set_flag(int* act, int j, int v)
{
    if (threadIdx.x == 0) act[j] = v;
}

void launch_set_flag(int* act, int j, int v, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, st, act, j, v);
}

// masked element-wise kernels: field j = blockIdx.y of nrhs fields of n nodes
template <typename T>
__global__ void k_masked_copy(const T* __restrict__ src, const uint8_t* __restrict__ mask,
                              T* __restrict__ dst, long n)
{
    const long off = blockIdx.y * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        dst[off + i] = mask[i] ? src[off + i] : T(0);
}

template <typename T>
void launch_masked_copy(const T* src, const uint8_t* mask, T* dst, long n, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL((k_masked_copy<T>), dim3(ew_blocks(n), nrhs), dim3(256), 0, st, src, mask,
                       dst, n);
}
template void launch_masked_copy<double>(const double*, const uint8_t*, double*, long, int,
                                         hipStream_t);
template void launch_masked_copy<float>(const float*, const uint8_t*, float*, long, int,
                                        hipStream_t);

__global__ void k_sub_masked(const double* __restrict__ a, const double* __restrict__ b,
                             const uint8_t* __restrict__ mask, double* __restrict__ out, long n)
{
    const long off = blockIdx.y * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        out[off + i] = mask[i] ? a[off + i] - b[off + i] : 0.0;
}

void launch_sub_masked(const double* a, const double* b, const uint8_t* mask, double* out, long n,
                       int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(k_sub_masked, dim3(ew_blocks(n), nrhs), dim3(256), 0, st, a, b, mask, out,
                       n);
}

__global__ void k_select(const uint8_t* __restrict__ mask, const double* __restrict__ a,
                         const double* __restrict__ b, double* __restrict__ out, long n)
{
    const long off = blockIdx.y * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        out[off + i] = mask[i] ? a[off + i] : b[off + i];
}

void launch_select(const uint8_t* mask, const double* a, const double* b, double* out, long n,
                   int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(k_select, dim3(ew_blocks(n), nrhs), dim3(256), 0, st, mask, a, b, out, n);
}

// Coefficient rows of another K-type product (App. C): rows [0, nba) are
// sqrt(ck) b^a, the row after them sqrt(cm) b^0, in the [row][s][nn] layout
// of b^a.
__global__ void k_op_rows(const double* __restrict__ ba, const double* __restrict__ b0, long nba,
                          long total, double wk, double wm, const double* __restrict__ wnode,
                          long nn, double* __restrict__ o64, float* __restrict__ o32)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
         i += (long)gridDim.x * blockDim.x) {
        double v;
        if (i < nba) {
            v = wk * ba[i];
        } else {
            const long j = i - nba;  // [s][nn]: node j % nn
            v = (wnode ? sqrt(wnode[j % nn]) : wm) * b0[j];
        }
        o64[i] = v;
        o32[i] = (float)v;
    }
}

void launch_op_rows(const Ctx& c, double ck, double cm, double* o64, float* o32, hipStream_t st,
                    const double* wnode)
{
    const long per = (long)c.s * c.nn;
    const long nba = ck > 0.0 ? (long)c.dim * per : 0;
    const long total = nba + (cm > 0.0 ? per : 0);
    hipLaunchKernelGGL(k_op_rows, dim3(ew_blocks(total)), dim3(256), 0, st, c.ba_64, c.b0_64, nba,
                       total, sqrt(ck), sqrt(cm), wnode, c.nn, o64, o32);
}

__global__ void k_pow_scaled(const double* __restrict__ u, double kappa, int cube,
                             double* __restrict__ out, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const double v = u[i];
        out[i] = cube ? kappa * v * v * v : kappa * v * v;
    }
}

void launch_pow_scaled(const double* u, double kappa, int pw, double* out, long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_pow_scaled, dim3(ew_blocks(n)), dim3(256), 0, st, u, kappa,
                       pw == 3 ? 1 : 0, out, n);
}

// Line search of the nonlinear CG (App. B.3, Alg B.3): the nonlinear part of
// phi'(alpha) = R(d + alpha p) . p is a nodal sum that is a cubic polynomial
// in alpha, s(alpha) = c0 + c1 alpha + c2 alpha^2 + c3 alpha^3, over the
// domain nodes (chi), so one pass gives its four coefficients:
//   kind 0, N(u) = kappa u^3, fields u = N d, w = N p: V kappa (u + alpha w)^3 w,
//     c0 = sum V kappa u^3 w, c1 = 3 sum V kappa u^2 w^2, c2 = 3 sum V kappa u w^3,
//     c3 = sum V kappa w^4;
//   kind 1, N(g) = (1 + kappa |g|^2) g, fields g = B d, h = B p (dim
//     components nn apart): V (1 + kappa |g + alpha h|^2)(g + alpha h) . h with
//     gg = |g|^2, gh = g . h, hh = |h|^2,
//     c0 = sum V (1 + kappa gg) gh, c1 = sum V [(1 + kappa gg) hh + 2 kappa gh^2],
//     c2 = 3 sum V kappa gh hh, c3 = sum V kappa hh^2.
// Per-block partials of c_j go to part[j kRedBlocks + b].
__global__ __launch_bounds__(kRedThreads) void k_ls_poly(int kind, int dim, const double* __restrict__ a,
                                                         const double* __restrict__ b,
                                                         const double* __restrict__ vol,
                                                         const uint8_t* __restrict__ chi, double kappa,
                                                         long n, double* __restrict__ part)
{
    __shared__ double sh[16];
    double c[4] = {0.0, 0.0, 0.0, 0.0};
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        if (!chi[i]) continue;
        const double v = vol[i];
        if (kind == 0) {
            const double u = a[i], w = b[i], vk = v * kappa;
            c[0] += vk * u * u * u * w;
            c[1] += 3.0 * vk * u * u * w * w;
            c[2] += 3.0 * vk * u * w * w * w;
            c[3] += vk * w * w * w * w;
        } else {
            double gg = 0.0, gh = 0.0, hh = 0.0;
            for (int k = 0; k < dim; ++k) {
                const double g = a[(long)k * n + i], h = b[(long)k * n + i];
                gg += g * g;
                gh += g * h;
                hh += h * h;
            }
            const double f = 1.0 + kappa * gg;
            c[0] += v * f * gh;
            c[1] += v * (f * hh + 2.0 * kappa * gh * gh);
            c[2] += 3.0 * v * kappa * gh * hh;
            c[3] += v * kappa * hh * hh;
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double t = block_sum(c[j], sh);
        if (threadIdx.x == 0) part[(long)j * kRedBlocks + blockIdx.x] = t;
    }
}

void launch_ls_poly(int kind, int dim, const double* a, const double* b, const double* vol,
                    const uint8_t* chi, double kappa, long n, double* part, hipStream_t st)
{
    hipLaunchKernelGGL(k_ls_poly, dim3(red_blocks(n)), dim3(kRedThreads), 0, st, kind, dim, a, b, vol,
                       chi, kappa, n, part);
}

__global__ void k_lincomb_masked(const double* __restrict__ a, double wa,
                                 const double* __restrict__ b, double wb,
                                 const double* __restrict__ cc, const uint8_t* __restrict__ mask,
                                 double* __restrict__ out, long n)
{
    const long off = blockIdx.y * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        double v = wa * a[off + i];
        if (b) v += wb * b[off + i];
        if (cc) v += cc[off + i];
        out[off + i] = mask[i] ? v : 0.0;
    }
}

void launch_lincomb_masked(const double* a, double wa, const double* b, double wb, const double* cc,
                           const uint8_t* mask, double* out, long nn, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(k_lincomb_masked, dim3(ew_blocks(nn), nrhs), dim3(256), 0, st, a, wa, b, wb,
                       cc, mask, out, nn);
}

__global__ void k_explicit_update(double* __restrict__ x, const double* __restrict__ kx,
                                  const double* __restrict__ c0, const double* __restrict__ ml,
                                  double w, const uint8_t* __restrict__ mask, long n)
{
    const long off = blockIdx.y * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        x[off + i] = mask[i] ? x[off + i] + (c0[off + i] - w * kx[off + i]) / ml[i] : 0.0;
}

void launch_explicit_update(double* x, const double* kx, const double* c0, const double* ml,
                            double w, const uint8_t* mask, long nn, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(k_explicit_update, dim3(ew_blocks(nn), nrhs), dim3(256), 0, st, x, kx, c0,
                       ml, w, mask, nn);
}

__global__ void k_check_positive(const double* __restrict__ v, const uint8_t* __restrict__ mask,
                                 long n, int* flag)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        if (mask[i] && !(v[i] > 0.0)) atomicOr(flag, 1);
}

void launch_check_positive(const double* v, const uint8_t* mask, long nn, int* flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_positive, dim3(ew_blocks(nn)), dim3(256), 0, st, v, mask, nn, flag);
}

__global__ void k_to32(const double* __restrict__ a, float* __restrict__ out, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        out[i] = (float)a[i];
}

void launch_to32(const double* a, float* out, long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_to32, dim3(ew_blocks(n)), dim3(256), 0, st, a, out, n);
}

__global__ void k_add32to64_reset(double* __restrict__ x, float* __restrict__ c, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        x[i] += (double)c[i];
        c[i] = 0.0f;
    }
}

void launch_add32to64_reset(double* x, float* c, long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_add32to64_reset, dim3(ew_blocks(n)), dim3(256), 0, st, x, c, n);
}

__global__ void k_add_reset64(double* __restrict__ x, double* __restrict__ c, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        x[i] += c[i];
        c[i] = 0.0;
    }
}

void launch_add_reset64(double* x, double* c, long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_add_reset64, dim3(ew_blocks(n)), dim3(256), 0, st, x, c, n);
}

}  // namespace fcrkpm
