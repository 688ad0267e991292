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
    int W;        // lines per tile (one workgroup), a power of two
    int wl;       // log2 W
    int contig;   // st == 1
};

// One term of a separable pass: output real field `out` gets
// coef * (input real field `in`) convolved along the axis with t_e, the
// 1D kernel-times-monomial array of exponent e (Sec 5.3, Eq 77-78).
constexpr int kMaxSepOut = 36;
constexpr int kMaxSepTerms = 40;
struct SepTerm {
    int32_t out, in, e, pad;
    double coef;
};
struct SepProg {
    int nin, nout;                 // real fields in / out
    int ostart[kMaxSepOut + 1];    // terms of output f: [ostart[f], ostart[f+1])
    SepTerm t[kMaxSepTerms];
};

// Programs of one monomial set over the active axes: part 1 maps the prefix
// set P_{j-1} to P_j along axis j, part 2 maps P_j back to P_{j-1}.
struct SepPlan {
    int k = 0;                    // active axes
    SepProg p1[3], p2[3];         // host copies (sizes, LDS planning)
    const SepProg* d1[3] = {};    // device copies read by the kernels
    const SepProg* d2[3] = {};
    int size[3] = {0, 0, 0};      // |P_j| real fields
    int maxpairs = 0;             // largest pair count of P_0 .. P_{k-2}
};

// Coefficients shared by the interior nodes (class 1): nodes whose support
// neighbourhood lies in the domain have the full-grid moment matrix, so b^a
// and V agree with those of the first such node (checked to 1e-12 of max |b|).
constexpr int kMaxNodeConst = 30;  // dim * s up to the quadratic basis in 3D
struct NodeConst {
    double b[kMaxNodeConst];       // coefficient rows of the product, row-major (b^a_q for K)
    double v;                      // V
    double bmax;                   // max |b|; negative: no interior node
};

// Pointwise data of one K-type product, E_p = V sum_rows c_p (c . D): the
// stiffness K takes the rows b^a (Eq 90-91), the consistent mass the single
// row b^0 (Eq C.8, C.11) and c_m M + c_k K the rows sqrt(c_k) b^a followed by
// sqrt(c_m) b^0.  The context holds the set in use; the others wait here and
// are swapped in for the products they serve.
struct OpSet {
    int krows = 0;
    double* ba_64 = nullptr;            // [krows][s][nn]
    float* ba_32 = nullptr;
    uint8_t* cls = nullptr;
    long ncls2 = 0;
    double cint64[kMaxNodeConst + 1] = {};
    float cint32[kMaxNodeConst + 1] = {};
    uint2* nbits[2] = {};
    float reg_mi[10] = {};
    uint32_t* noff[2] = {};
    float* nrec[2] = {};
    long nload[2] = {-1, -1};
    NodeConst nconst = {};
    void* sym = nullptr;                // line-constant records of this set's rows
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
    double* area64 = nullptr;           // boundary areas A of the flux nodes (App. A), or NULL
    float* area32 = nullptr;
    double* b0_64 = nullptr;            // [s][nn]
    double* ba_64 = nullptr;            // [krows][s][nn]: rows of the K-type product in use
    float* b0_32 = nullptr;
    float* ba_32 = nullptr;
    cplx<double>* tw64[3] = {};         // twiddles per axis
    cplx<float>* tw32[3] = {};
    cplx<double>* spec64[3] = {};       // kernel spectra per axis, exponents 0..2n
    cplx<float>* spec32[3] = {};
    float* rtab32[3] = {};              // per axis [2][n]: Re T_0 / n, Im T_1 / n (register passes)
    int krows = 0;                      // coefficient rows of the K-type product in use (dim for K)
    OpSet* mass_set = nullptr;          // consistent mass (built on first use)
    OpSet* shift_set = nullptr;         // c_m M + c_k K of the last implicit time step
    double shift_w[2] = {0.0, 0.0};     // its (c_m, c_k)
    double pw_kappa = 0.0;              // kappa of the gradient nonlinearity (SEP_PW_KN middle passes)
    OpSet* jac_set = nullptr;           // K + N^T diag(w V) N of the last Newton step
    bool use_regpath = true;            // register-resident passes where they apply
    uint8_t* cls = nullptr;             // node class: 0 outside the domain, 1 interior, 2 other
    long ncls2 = 0;                     // class-2 nodes
    double cint64[kMaxNodeConst + 1] = {};  // interior b^a (a-major) and V
    float cint32[kMaxNodeConst + 1] = {};
    uint2* nbits[2] = {};               // register path: node-class bits per middle-pass lane, per layout
    float reg_mi[10] = {};              // register path: M = V B^T B of the interior nodes
    uint32_t* noff[2] = {};             // register path: first record of each lane, per layout
    float* nrec[2] = {};                // register path: coefficient records (0: interior), per layout
    int reg_layout = 0;                 // register path: line layout (0: 8 lanes, 1: 16 lanes)
    int reg_tpw = 1;                    // register path: tiles per workgroup (1 or 2)
    float tune_ms[4] = {};              // register path: measured K product per variant
                                        // (layout + 2 (tiles - 1)); 0: untimed
    long nload[2] = {-1, -1};           // register path: middle-pass elements reading the arrays
    bool prof_dot = false;              // the sampled K product carries the fused p.q
    bool prof_pupd = false;             // ... and the fused direction update
    NodeConst nconst = {};              // values of the interior nodes
    // workspace: two slots of SepPlan::maxpairs complex fields per precision
    // and right-hand side (cap_work of them)
    cplx<double>* work64 = nullptr;
    cplx<float>* work32 = nullptr;
    // real vectors for the solvers
    double* v64 = nullptr;              // 6 FP64 vectors of cap_rhs fields
    float* v32 = nullptr;               // 5 FP32 vectors of cap_rhs fields
    double* partial = nullptr;          // reduction partials (2 x cap_rhs x kRedBlocks)
    double* partial_wide = nullptr;     // p.q partials of a last pass with more workgroups
                                        // than kRedBlocks (cap_rhs x reg_dot_slots)
    double* scal = nullptr;             // device scalars (cap_rhs x kScal)
    double* hscal = nullptr;            // pinned host mirror (2 poll slots + 1 read slot)
    int* act = nullptr;                 // per right-hand side: still iterating
    int cap_rhs = 0;                    // right-hand sides the solver buffers hold
    int cap_work = 0;                   // right-hand sides the pass workspace holds
    bool capturing = false;             // a graph capture is recording this context's work
    hipStream_t aux = nullptr;          // stream of this problem inside a batched solve
    int* dflag = nullptr;               // device int flags
    void* prof = nullptr;               // kernel-duration sampler (measurement only)
    bool prof_on = false;
    int prof_rhs = 1;                   // right-hand sides of the launch being sampled
    bool use_graphs = true;             // replay CG blocks from captured graphs
    SepPlan basis_plan;                 // basis monomials (Alg 2-4)
    SepProg* dprog = nullptr;           // device copies of the pass programs
    int lds_budget = 65536;             // LDS bytes one workgroup may use
    void* scratch = nullptr;            // device address of this device's static scratch array
                                        // (fcrkpm_apply_noalloc), taken at setup
    int sep_wcap[2] = {16, 16};         // LDS-tiled passes: most lines per workgroup (FP32, FP64),
                                        // chosen at setup by timing K products
    bool tune_cached = false;           // the autotuner's choices came from its cache file
    void* sym = nullptr;                // register path: line-constant middle pass of K (regpass.hip)
    bool use_sym = true;                // use it where it applies
    double* rtab64[3] = {};             // per axis [3][n]: Re T_0 / n, Im T_1 / n, Re T_2 / n (FP64)
};

constexpr int kRedBlocks = 1024;   // reduction partials per right-hand side (at most)
constexpr int kRedThreads = 256;
constexpr int kScal = 8;           // device scalars per right-hand side

// Right-hand sides of one launch (blockIdx.y) and the byte strides between
// their input, output and source fields.
struct RhsBatch {
    int n = 1;
    long in_bytes = 0, out_bytes = 0, src_bytes = 0;
};

// ------------------------------------------------------------- launchers
// separable passes (sepconv.hip); load/store and pointwise modes:
enum { SEP_LD_PAIRS = 0, SEP_LD_REAL = 1, SEP_LD_CHI = 2 };
enum { SEP_ST_PAIRS = 0, SEP_ST_REAL = 1 };
enum { SEP_PW_K = 0, SEP_PW_UH = 1, SEP_PW_LOAD = 2, SEP_PW_KN = 3 };  // KN: K with A scaled by 1 + kappa |A|^2

template <typename T, typename Tio>
void launch_sep_pass(const Ctx& c, int a, const SepProg& pr, const SepProg* dpr, int ldm,
                     const void* in,
                     const uint8_t* mask_in, int stm, void* out, const uint8_t* mask_out,
                     double* dot_part, const void* dot_with, hipStream_t st,
                     const RhsBatch& rb = RhsBatch{});

template <typename T, typename Tio>
void launch_sep_mid(const Ctx& c, int a, const SepProg& pr1, const SepProg* dpr1,
                    const SepProg& pr2, const SepProg* dpr2, int pw, int ldm,
                    const void* in, const uint8_t* mask_in, int stm, void* out,
                    const uint8_t* mask_out, const void* src, const T* b0, const T* ba,
                    const T* vol, double* dot_part, const void* dot_with, hipStream_t st,
                    const RhsBatch& rb = RhsBatch{});

// Register-resident passes of the K-type products (regpass.hip) for cubic 3D
// boxes of the register-path lengths.  `prof` brackets the five launches (x,
// y, middle z, y, x) for the kernel-duration sampler.
// Duration sampling of the register passes: for pass k (0..4) of a launch,
// events() counts the launch and either leaves both events null or hands out
// the pair that the launch itself records (hipExtLaunchKernelGGL), so the
// sampled span is the kernel's own, without separate event packets around it.
struct RegProf {
    const void* c = nullptr;
    void (*events_fn)(const void*, int, hipEvent_t*, hipEvent_t*) = nullptr;
    void events(int k, hipEvent_t* e0, hipEvent_t* e1) const
    {
        *e0 = *e1 = nullptr;
        if (events_fn) events_fn(c, k, e0, e1);
    }
};
// The CG direction update p = r + beta p that the first x pass of a K product
// may apply to its input p before transforming it (beta from the r.r partials
// of the previous x/r update, as the stand-alone update kernel computes it).
struct RegPupd {
    const float* r;
    const double* rr_part;
    int nrr;
    double* scal;
    int parity;
    const int* act;
};
bool reg_path_ok(const Ctx& c);
// 3D cube boxes of 32, 48, 80, 96 or 256 nodes per axis, linear basis: the
// register path with P x Q line layouts, which runs only with the
// line-constant middle pass (sym_active)
bool reg_gpq_ok(const Ctx& c);
// Line-constant middle pass of the register path (linear basis, K only): along
// every z line the pointwise matrix M = V B^T B is constant except at a few
// nodes near the ends of the z extent, so the middle pass applies the line's
// M in the spectral domain and corrects those nodes directly.  sym_build
// analyses the coefficient rows in use (K's) and keeps the state in c.sym
// when the geometry allows it; sym_active tells whether the current product
// can use it; sym_release frees it.
void sym_build(Ctx& c, hipStream_t st);
bool sym_active(const Ctx& c);
void sym_release(Ctx& c);
void sym_release_state(void*& sym);
// algorithmic bytes of one launch of that middle pass per right-hand side
double sym_pass_bytes(const Ctx& c, int elem_bytes);
// The FP64 K product on the register path (linear basis, 32^3, 48^3, 64^3,
// 128^3 or 256^3 boxes with the line-constant middle pass): reg_path64_ok
// tells whether it applies; with dot_part the last pass also leaves the
// per-workgroup partials of out . dot_with (reg_path64_blocks of them per
// right-hand side, kRedBlocks or reg_dot_slots apart).
bool reg_path64_ok(const Ctx& c);
// The force of the gradient nonlinearity, the implicit gradient B d, u^h and the
// load f^r on the FP64 register path (line-constant middle passes; the force
// with the nonlinearity between its halves); reg_kn_ok builds their records on
// first use and tells whether the path serves this problem.  One field per
// launch.
enum { RK_FORCE = 0, RK_GRAD = 1, RK_UH = 2, RK_LOAD = 3 };
bool reg_kn_ok(const Ctx& c, hipStream_t st);
void launch_reg_kn(const Ctx& c, const double* in, double* out, double kappa, int mode, hipStream_t st);
long reg_path64_blocks(const Ctx& c);
void launch_reg_k64(const Ctx& c, const double* in, double* out, const uint8_t* mask, int nrhs,
                    double* dot_part, const double* dot_with, hipStream_t st, const RegProf& prof);
int reg_path_blocks(const Ctx& c);
// partial slots per right-hand side of the register path's last-pass dot:
// kRedBlocks where every variant's last pass fits them, else the most
// workgroups any variant launches (no layout holds fewer than 16 lines per
// workgroup); the dot partials of a launch with more workgroups than
// kRedBlocks lie reg_dot_slots apart between right-hand sides
long reg_dot_slots(const Ctx& c);
int reg_layouts(const Ctx& c);
bool reg_variant_ok(const Ctx& c, int v);
long reg_bits_words(const Ctx& c, int layout);
void launch_reg_bits(const Ctx& c, int layout, const uint8_t* cls, uint2* bits, uint32_t* count,
                     unsigned long long* nload, hipStream_t st);
void launch_reg_recs(const Ctx& c, int layout, const uint2* bits, const uint32_t* off,
                     float* rec, hipStream_t st);
int reg_record_floats(const Ctx& c);
void launch_reg_k(const Ctx& c, const float* in, float* out, const uint8_t* mask, int nrhs,
                  double* dot_part, const float* dot_with, hipStream_t st, const RegProf& prof,
                  const RegPupd* pu = nullptr);

// throws the library's FCRKPM_ERR_UNSUPPORTED status with this message
[[noreturn]] void raise_unsupported(const char* msg);

// LDS bytes the passes of a plan need at the tile widths they will use
size_t sep_lds_need(const Ctx& c, const SepPlan& sp, int elem_bytes);


void launch_free_mask(const uint8_t* chi, const uint8_t* dir, uint8_t* freem, int* bad, long nn,
                      hipStream_t st);
void launch_axis_extent(const Ctx& c, const uint8_t* chi, int* occ, hipStream_t st);
void launch_moment_solve(const Ctx& c, const cplx<double>* G, int* bad, hipStream_t st);
void launch_first_interior(const Ctx& c, int* ref, hipStream_t st);
void launch_node_class(const Ctx& c, const NodeConst& ref, uint8_t* cls, hipStream_t st);
void launch_vol(const uint8_t* chi, const double* vol_in, double hv, double* vol64, float* vol32,
                long nn, hipStream_t st);
void launch_mask_to_double(const uint8_t* m, double* out, long nn, hipStream_t st);
void launch_check_finite(const double* x, long nn, int* flag, hipStream_t st);
// rows of another K-type product: sqrt(ck) b^a (when ck > 0), then sqrt(cm) b^0 (when cm > 0),
// the latter with sqrt(wnode) per node in place of sqrt(cm) when wnode is given
void launch_op_rows(const Ctx& c, double ck, double cm, double* o64, float* o32, hipStream_t st,
                    const double* wnode = nullptr);
// out = kappa u^pw (pw 2 or 3) over n values
void launch_pow_scaled(const double* u, double kappa, int pw, double* out, long n, hipStream_t st);
// coefficients of the nonlinear part of the nonlinear CG's line-search
// derivative, a cubic in the step (kind 0: kappa u^3 with a = N d, b = N p;
// kind 1: (1 + kappa |g|^2) g with a = B d, b = B p, dim fields each):
// per-block partials of c_j in part[j kRedBlocks + b], j = 0..3
void launch_ls_poly(int kind, int dim, const double* a, const double* b, const double* vol,
                    const uint8_t* chi, double kappa, long n, double* part, hipStream_t st);
// out = mask ? wa a + wb b + c : 0 (b and c may be NULL) over nrhs fields
void launch_lincomb_masked(const double* a, double wa, const double* b, double wb, const double* cc,
                           const uint8_t* mask, double* out, long nn, int nrhs, hipStream_t st);
// forward Euler with the lumped mass: x = mask ? x + (c0 - w kx) / ml : 0
void launch_explicit_update(double* x, const double* kx, const double* c0, const double* ml,
                            double w, const uint8_t* mask, long nn, int nrhs, hipStream_t st);
// flag |= 1 where mask and !(v > 0)
void launch_check_positive(const double* v, const uint8_t* mask, long nn, int* flag, hipStream_t st);

// CG / vector kernels (deterministic two-stage reductions), batched over
// nrhs right-hand sides: vectors of rhs j start at j*n, its scalars at
// j*kScal, its reduction partials at j*kRedBlocks; act[j] == 0 freezes it.
int red_blocks(long n);
template <typename T>
void launch_dot_partial(const T* a, const T* b, long n, int nrhs, double* part, const int* act,
                        hipStream_t st);
void launch_reduce_to(const double* part, long n, int nrhs, double* dst, hipStream_t st);
// dst[j * kRedBlocks] = the sum of nb partials at part + j * stride, in the
// fixed order of the other reductions
void launch_reduce_wide(const double* part, int nb, long stride, int nrhs, double* dst, hipStream_t st);
template <typename T>
void launch_cg_xr(T* x, T* r, const T* p, const T* q, long n, int nrhs, const double* pq_part,
                  int npq, double* scal, int parity, double* rr_part, const int* act,
                  hipStream_t st);
template <typename T>
void launch_cg_p(T* p, const T* r, long n, int nrhs, const double* rr_part, double* scal,
                 int parity, const int* act, hipStream_t st);
void launch_set_scalar(double* scal, int idx, double v, int nrhs, hipStream_t st);
void launch_set_flag(int* act, int j, int v, hipStream_t st);
template <typename T>
void launch_masked_copy(const T* src, const uint8_t* mask, T* dst, long n, int nrhs,
                        hipStream_t st);
void launch_sub_masked(const double* a, const double* b, const uint8_t* mask, double* out,
                       long n, int nrhs, hipStream_t st);
void launch_select(const uint8_t* mask, const double* a, const double* b, double* out, long n,
                   int nrhs, hipStream_t st);
// flat over all elements (n = nodes * nrhs)
void launch_to32(const double* a, float* out, long n, hipStream_t st);
void launch_add32to64_reset(double* x, float* c, long n, hipStream_t st);
void launch_add_reset64(double* x, double* c, long n, hipStream_t st);

}  // namespace fcrkpm
