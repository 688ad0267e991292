// fcrkpm_impl.hpp -- host-side context and the launchers shared by the
// library's translation units (kernels.hip, fcrkpm.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <string>
#include <vector>

#include "fft_core.hpp"

namespace fcrkpm {

constexpr int kMaxS = 10;         // basis size: 3D quadratic
constexpr int kMaxMono = 35;      // monomials of degree <= 2n in 3D, n = 2
constexpr int kMaxTerms = 48;     // spectral terms of one convolution pass
constexpr int kMaxIO = 20;        // fields on the multi side of a convolution pass

// Geometry of the line transforms along one axis.
struct AxisGeom {
    int L;        // line length (box nodes on the axis)
    long st;      // element stride of the axis
    long nlines;  // lines in a field (nodes / L)
    int W;        // lines per tile (one workgroup)
    int contig;   // st == 1
};

// One spectral term: coef * F(H_m)(k), with F(H_m) the separable spectrum of
// the kernel-times-monomial array of monomial m (Sec 5.3, Eq 77-78).
struct SpecTerm {
    int mono;
    double re, im;
};

// Spectral program of one convolution pass: either one input and nio outputs
// (output j gets sum of terms [start[j], start[j+1]) times the input spectrum)
// or nio inputs and one output (sum over inputs l of terms times input l).
struct ConvProg {
    int nio;
    int multi_in;                 // 0: 1 -> nio, 1: nio -> 1
    int start[kMaxIO + 1];
    SpecTerm term[kMaxTerms];
    int8_t mexp[kMaxMono][3];     // monomial exponents per axis
};

// Per-axis spectral tables: spec[a][e][k] = sum_o o^e phi1(|o| / at_a) e^{-2 pi i k o / n_a}.
struct SpecTables {
    const void* base[3];  // complex<T> tables, e-major, n_a entries per exponent
};

struct Ctx {
    int dim = 0;
    int n[3] = {1, 1, 1};
    double h[3] = {1, 1, 1};
    double at[3] = {0, 0, 0};
    int m[3] = {0, 0, 0};
    int degree = 1;
    int s = 0;
    int ex[kMaxS][3] = {};
    int nmono2 = 0;                     // monomials of degree <= 2n
    int ex2[kMaxMono][3] = {};
    long nn = 0;
    int naxes = 0;
    int axes[3] = {0, 0, 0};            // active axes (n > 1), ascending
    LinePlan plan[3] = {};
    std::string err;

    // device data (owned)
    uint8_t* chi = nullptr;             // domain mask
    uint8_t* freem = nullptr;           // chi_Omega
    uint8_t* dirm = nullptr;            // chi_Gamma_g
    double* vol64 = nullptr;
    float* vol32 = nullptr;
    double* b0_64 = nullptr;            // [s][nn]
    double* ba_64 = nullptr;            // [dim][s][nn]
    float* b0_32 = nullptr;
    float* ba_32 = nullptr;
    cplx<double>* tw64[3] = {};         // twiddles per axis
    cplx<float>* tw32[3] = {};
    cplx<double>* spec64[3] = {};       // kernel spectra per axis, exponents 0..2n
    cplx<float>* spec32[3] = {};
    // workspace: (npairs + 1) complex fields per precision
    int npairs = 0;
    cplx<double>* work64 = nullptr;
    cplx<float>* work32 = nullptr;
    // real vectors for the solvers
    double* v64 = nullptr;              // 6 FP64 vectors
    float* v32 = nullptr;               // 5 FP32 vectors
    double* partial = nullptr;          // reduction partials (2 x kRedBlocks)
    double* scal = nullptr;             // device scalars
    double* hscal = nullptr;            // pinned host mirror
    int* dflag = nullptr;               // device int flags
    void* prof = nullptr;               // kernel-duration sampler (measurement only)
    bool prof_on = false;
    ConvProg prog_fwd;                  // d -> D_q pairs (H_q^a)
    ConvProg prog_bwd;                  // E_p pairs -> f (conj-reflected H_p^a)
};

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// ------------------------------------------------------------- launchers
AxisGeom axis_geom(const Ctx& c, int a, int elem_bytes);

template <typename T>
void launch_line_pass(const Ctx& c, int a, int dir, cplx<T>* data, int nfields, long fstride,
                      hipStream_t st);

template <typename T>
void launch_conv_pass(const Ctx& c, int a, const ConvProg& prog, const cplx<T>* in, cplx<T>* out,
                      hipStream_t st);

template <typename Tin, typename T>
void launch_pack(const Tin* d, const uint8_t* mask, cplx<T>* U, long nn, hipStream_t st);

template <typename T, typename Tout>
void launch_unpack_re(const cplx<T>* R, const uint8_t* mask, Tout* out, long nn, hipStream_t st);

template <typename T>
void launch_pointwise_k(const Ctx& c, cplx<T>* DE, const T* ba, const T* vol, hipStream_t st);

template <typename T, typename Tout>
void launch_pointwise_uh(const Ctx& c, const cplx<T>* D, const T* b0, const T* vol, Tout* out,
                         hipStream_t st);

template <typename Tin, typename T>
void launch_pointwise_load(const Ctx& c, const Tin* r, const T* b0, const T* vol, cplx<T>* E,
                           hipStream_t st);

void launch_chi_pack(const uint8_t* chi, cplx<double>* U, long nn, hipStream_t st);
void launch_free_mask(const uint8_t* chi, const uint8_t* dir, uint8_t* freem, int* bad, long nn,
                      hipStream_t st);
void launch_axis_extent(const Ctx& c, const uint8_t* chi, int* occ, hipStream_t st);
void launch_moment_solve(const Ctx& c, const cplx<double>* G, int* bad, hipStream_t st);
void launch_vol(const uint8_t* chi, const double* vol_in, double hv, double* vol64, float* vol32,
                long nn, hipStream_t st);
void launch_mask_to_double(const uint8_t* m, double* out, long nn, hipStream_t st);
void launch_check_finite(const double* x, long nn, int* flag, hipStream_t st);

// CG / vector kernels (deterministic two-stage reductions)
template <typename T>
void launch_dot_partial(const T* a, const T* b, long n, double* part, hipStream_t st);
void launch_reduce_to(const double* part, double* dst, hipStream_t st);
template <typename T>
void launch_cg_xr(T* x, T* r, const T* p, const T* q, long n, const double* pq_part,
                  double* scal, int parity, double* rr_part, hipStream_t st);
template <typename T>
void launch_cg_p(T* p, const T* r, long n, const double* rr_part, double* scal, int parity,
                 hipStream_t st);
template <typename T>
void launch_masked_copy(const T* src, const uint8_t* mask, T* dst, long n, hipStream_t st);
void launch_residual64(const double* b, const double* kx, const uint8_t* mask, double* r, long n,
                       hipStream_t st);
void launch_scale_to32(const double* r, const double* scal, int idx, float* out, long n,
                       hipStream_t st);
void launch_axpy32to64(double* x, const float* c, const double* scal, int idx, long n,
                       hipStream_t st);
void launch_sub_masked(const double* a, const double* b, const uint8_t* mask, double* out,
                       long n, hipStream_t st);
void launch_select(const uint8_t* mask, const double* a, const double* b, double* out, long n,
                   hipStream_t st);
void launch_mul(const double* a, const double* b, double* out, long n, hipStream_t st);

}  // namespace fcrkpm
