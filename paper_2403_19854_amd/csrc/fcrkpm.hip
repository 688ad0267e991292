// fcrkpm.hip -- host side of the C ABI declared in include/fcrkpm.h: argument
// checks, plans and spectral tables, the convolution pipelines of Alg 1-4,
// the CG drivers (FP64, and FP32 inside FP64 iterative refinement) and the
// adjoint solve.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <string>
#include <vector>

#include "../../include/fcrkpm.h"
#include "fcrkpm_impl.hpp"

using namespace fcrkpm;

struct fcrkpm_ctx {
    Ctx c;
};

namespace {

thread_local std::string g_setup_err;

struct HipFail {
    hipError_t e;
    const char* what;
};

#define HIPCHK(expr)                                  \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) throw HipFail{e_, #expr}; \
    } while (0)

struct ArgFail {
    fcrkpm_status st;
    std::string msg;
};

[[noreturn]] void fail(fcrkpm_status st, const std::string& msg) { throw ArgFail{st, msg}; }

// ------------------------------------------------------ kernel-duration sampler
// For each kernel kind, HIP events bracket the first kProfCap launches after
// sampling starts; every launch is counted together with its algorithmic
// bytes (what the launch must read and write, from the array sizes).
enum Kind {
    KD_LINE_FWD_X, KD_LINE_FWD_Y, KD_LINE_FWD_Z, KD_LINE_INV_X, KD_LINE_INV_Y, KD_LINE_INV_Z,
    KD_CONV_FWD, KD_CONV_BWD, KD_PACK, KD_UNPACK, KD_POINT_K, KD_POINT_UH, KD_POINT_LOAD,
    KD_NKINDS
};
const char* const kKindNames[KD_NKINDS] = {
    "line_pass_fwd_x", "line_pass_fwd_y", "line_pass_fwd_z", "line_pass_inv_x", "line_pass_inv_y",
    "line_pass_inv_z", "conv_pass_1_to_pairs", "conv_pass_pairs_to_1", "pack", "unpack_re",
    "pointwise_k", "pointwise_uh", "pointwise_load"};
constexpr int kProfCap = 64;

struct ProfKind {
    long launches = 0;
    double bytes = 0.0;
    int nrec = 0;
    hipEvent_t ev[2 * kProfCap];
};

struct Prof {
    ProfKind k[KD_NKINDS];
};

struct ProfScope {
    Prof* p;
    int kind;
    hipStream_t st;
    bool rec = false;
    ProfScope(Ctx& c, int kind_, double bytes, hipStream_t st_)
        : p(c.prof_on ? (Prof*)c.prof : nullptr), kind(kind_), st(st_)
    {
        if (!p) return;
        ProfKind& k = p->k[kind];
        ++k.launches;
        k.bytes += bytes;
        if (k.nrec < kProfCap) {
            (void)hipEventRecord(k.ev[2 * k.nrec], st);
            rec = true;
        }
    }
    ~ProfScope()
    {
        if (!rec) return;
        ProfKind& k = p->k[kind];
        (void)hipEventRecord(k.ev[2 * k.nrec + 1], st);
        ++k.nrec;
    }
};

template <typename T>
T* dalloc(size_t count)
{
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) fail(FCRKPM_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    return reinterpret_cast<T*>(p);
}

template <typename T>
void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void release(Ctx& c)
{
    dfree(c.chi);
    dfree(c.freem);
    dfree(c.dirm);
    dfree(c.vol64);
    dfree(c.vol32);
    dfree(c.b0_64);
    dfree(c.ba_64);
    dfree(c.b0_32);
    dfree(c.ba_32);
    for (int a = 0; a < 3; ++a) {
        dfree(c.tw64[a]);
        dfree(c.tw32[a]);
        dfree(c.spec64[a]);
        dfree(c.spec32[a]);
    }
    dfree(c.work64);
    dfree(c.work32);
    dfree(c.v64);
    dfree(c.v32);
    dfree(c.partial);
    dfree(c.scal);
    dfree(c.dflag);
    if (c.hscal) (void)hipHostFree(c.hscal);
    c.hscal = nullptr;
    if (c.prof) {
        Prof* p = (Prof*)c.prof;
        for (auto& k : p->k)
            for (auto& e : k.ev) (void)hipEventDestroy(e);
        delete p;
        c.prof = nullptr;
    }
}

// Cubic B-spline profile (Sec 2.1, Eq 7) at z = |x| / a, in long double for the tables.
long double bspline(long double z)
{
    z = fabsl(z);
    if (z <= 0.5L) return 2.0L / 3.0L - 4.0L * z * z + 4.0L * z * z * z;
    if (z < 1.0L) {
        long double t = 1.0L - z;
        return 4.0L / 3.0L * t * t * t;
    }
    return 0.0L;
}

// Graded-lex monomials of total degree <= deg in `dim` variables (Eq 4 order).
int monomials(int dim, int deg, int (*ex)[3], int cap)
{
    int k = 0;
    for (int d = 0; d <= deg; ++d)
        for (int a = d; a >= 0; --a)
            for (int b = d - a; b >= 0; --b) {
                int cc = d - a - b;
                if (dim < 2 && b != 0) continue;
                if (dim < 3 && cc != 0) continue;
                if (k >= cap) return -1;
                ex[k][0] = a;
                ex[k][1] = b;
                ex[k][2] = cc;
                ++k;
            }
    return k;
}

bool make_plan(int n, LinePlan& p)
{
    p.n = n;
    p.nst = 0;
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
    auto push = [&](int rad) {
        if (p.nst >= kMaxStages) return false;
        p.rad[p.nst++] = rad;
        return true;
    };
    for (int i = 0; i < n8; ++i) if (!push(8)) return false;
    for (int i = 0; i < n4; ++i) if (!push(4)) return false;
    for (int i = 0; i < n2; ++i) if (!push(2)) return false;
    while (r % 3 == 0) {
        r /= 3;
        if (!push(3)) return false;
    }
    while (r % 5 == 0) {
        r /= 5;
        if (!push(5)) return false;
    }
    return r == 1;
}

int mono_of(const Ctx& c, int e0, int e1, int e2)
{
    for (int m = 0; m < c.nmono2; ++m)
        if (c.ex2[m][0] == e0 && c.ex2[m][1] == e1 && c.ex2[m][2] == e2) return m;
    return -1;
}

void prog_common(const Ctx& c, ConvProg& pg)
{
    memset(&pg, 0, sizeof(pg));
    for (int m = 0; m < c.nmono2; ++m)
        for (int a = 0; a < 3; ++a) pg.mexp[m][a] = (int8_t)c.ex2[m][a];
}

// Alg 2 first half / Alg 3: output pair j holds D_{2j} + i D_{2j+1} with
// D_q = (chi d) (*) H_q^a  (Eq 90, 94).  1/N of the inverse folded in.
void build_prog_fwd(const Ctx& c, ConvProg& pg)
{
    prog_common(c, pg);
    const double inv = 1.0 / (double)c.nn;
    int np = (c.s + 1) / 2, t = 0;
    pg.nio = np;
    pg.multi_in = 0;
    for (int j = 0; j < np; ++j) {
        pg.start[j] = t;
        int q = 2 * j;
        pg.term[t++] = SpecTerm{mono_of(c, c.ex[q][0], c.ex[q][1], c.ex[q][2]), inv, 0.0};
        if (q + 1 < c.s)
            pg.term[t++] = SpecTerm{mono_of(c, c.ex[q + 1][0], c.ex[q + 1][1], c.ex[q + 1][2]), 0.0, inv};
    }
    pg.start[np] = t;
}

// Alg 2 second half / Alg 4: input pair l = E_{2l} + i E_{2l+1}; the real part of
// the output is sum_p E_p (*) conj-reflected H_p^a  (Eq 55, 91, 92).  The
// reflected kernel has spectrum (-1)^deg(p) F(H_p^a); the pair uses
// H-bar_{2l} - i H-bar_{2l+1}.
void build_prog_bwd(const Ctx& c, ConvProg& pg)
{
    prog_common(c, pg);
    const double inv = 1.0 / (double)c.nn;
    int np = (c.s + 1) / 2, t = 0;
    pg.nio = np;
    pg.multi_in = 1;
    for (int l = 0; l < np; ++l) {
        pg.start[l] = t;
        int p = 2 * l;
        int dg = c.ex[p][0] + c.ex[p][1] + c.ex[p][2];
        double sg = (dg & 1) ? -1.0 : 1.0;
        pg.term[t++] = SpecTerm{mono_of(c, c.ex[p][0], c.ex[p][1], c.ex[p][2]), sg * inv, 0.0};
        if (p + 1 < c.s) {
            int dg1 = c.ex[p + 1][0] + c.ex[p + 1][1] + c.ex[p + 1][2];
            double sg1 = (dg1 & 1) ? -1.0 : 1.0;
            pg.term[t++] = SpecTerm{mono_of(c, c.ex[p + 1][0], c.ex[p + 1][1], c.ex[p + 1][2]), 0.0,
                                    -sg1 * inv};
        }
    }
    pg.start[np] = t;
}

// Alg 1: output pair j holds chi (*) (H_m phi) for monomials m = 2j, 2j+1 of
// degree <= 2n; M_pq reads monomial e_p + e_q (Eq 49, 80).
void build_prog_mom(const Ctx& c, ConvProg& pg)
{
    prog_common(c, pg);
    const double inv = 1.0 / (double)c.nn;
    int np = (c.nmono2 + 1) / 2, t = 0;
    pg.nio = np;
    pg.multi_in = 0;
    for (int j = 0; j < np; ++j) {
        pg.start[j] = t;
        pg.term[t++] = SpecTerm{2 * j, inv, 0.0};
        if (2 * j + 1 < c.nmono2) pg.term[t++] = SpecTerm{2 * j + 1, 0.0, inv};
    }
    pg.start[np] = t;
}

template <typename T>
cplx<T>* work_of(Ctx& c)
{
    if constexpr (sizeof(T) == 8) return c.work64;
    else return c.work32;
}

// Convolution of one complex field U into pair fields P (forward passes on all
// but the last axis, fused last-axis pass, inverse passes).
template <typename T>
void line_pass(Ctx& c, int a, int dir, cplx<T>* data, int nf, hipStream_t st)
{
    ProfScope ps(c, (dir > 0 ? KD_LINE_FWD_X : KD_LINE_INV_X) + a,
                 2.0 * nf * (double)c.nn * sizeof(cplx<T>), st);
    launch_line_pass<T>(c, a, dir, data, nf, c.nn, st);
}

template <typename T>
void conv_pass(Ctx& c, int a, const ConvProg& pg, const cplx<T>* in, cplx<T>* out, hipStream_t st)
{
    ProfScope ps(c, pg.multi_in ? KD_CONV_BWD : KD_CONV_FWD,
                 (1.0 + pg.nio) * (double)c.nn * sizeof(cplx<T>), st);
    launch_conv_pass<T>(c, a, pg, in, out, st);
}

template <typename T>
void conv_one_to_many(Ctx& c, const ConvProg& pg, cplx<T>* U, cplx<T>* P, hipStream_t st)
{
    const int k = c.naxes;
    for (int i = 0; i < k - 1; ++i) line_pass<T>(c, c.axes[i], +1, U, 1, st);
    conv_pass<T>(c, c.axes[k - 1], pg, U, P, st);
    for (int i = k - 2; i >= 0; --i) line_pass<T>(c, c.axes[i], -1, P, pg.nio, st);
}

template <typename T>
void conv_many_to_one(Ctx& c, const ConvProg& pg, cplx<T>* P, cplx<T>* U, hipStream_t st)
{
    const int k = c.naxes;
    for (int i = 0; i < k - 1; ++i) line_pass<T>(c, c.axes[i], +1, P, pg.nio, st);
    conv_pass<T>(c, c.axes[k - 1], pg, P, U, st);
    for (int i = k - 2; i >= 0; --i) line_pass<T>(c, c.axes[i], -1, U, 1, st);
}

template <typename T>
const T* b0_of(const Ctx& c)
{
    if constexpr (sizeof(T) == 8) return c.b0_64;
    else return c.b0_32;
}
template <typename T>
const T* ba_of(const Ctx& c)
{
    if constexpr (sizeof(T) == 8) return c.ba_64;
    else return c.ba_32;
}
template <typename T>
const T* vol_of(const Ctx& c)
{
    if constexpr (sizeof(T) == 8) return c.vol64;
    else return c.vol32;
}

// One operator on one field, precision T (Alg 2, 3, 4).
template <typename T>
void apply_one(Ctx& c, int op, const T* in, T* out, hipStream_t st)
{
    cplx<T>* U = work_of<T>(c);
    cplx<T>* P = U + c.nn;
    const double nn = (double)c.nn, ct = sizeof(cplx<T>), rt = sizeof(T);
    switch (op) {
        case FCRKPM_OP_K:
        case FCRKPM_OP_K_FULL: {
            const uint8_t* mk = (op == FCRKPM_OP_K) ? c.freem : c.chi;
            {
                ProfScope ps(c, KD_PACK, nn * (rt + 1 + ct), st);
                launch_pack<T, T>(in, mk, U, c.nn, st);
            }
            conv_one_to_many<T>(c, c.prog_fwd, U, P, st);
            {
                ProfScope ps(c, KD_POINT_K, nn * (2.0 * c.npairs * ct + (c.dim * c.s + 1) * rt), st);
                launch_pointwise_k<T>(c, P, ba_of<T>(c), vol_of<T>(c), st);
            }
            conv_many_to_one<T>(c, c.prog_bwd, P, U, st);
            {
                ProfScope ps(c, KD_UNPACK, nn * (ct + 1 + rt), st);
                launch_unpack_re<T, T>(U, mk, out, c.nn, st);
            }
            break;
        }
        case FCRKPM_OP_FR:
        case FCRKPM_OP_NT: {
            {
                ProfScope ps(c, KD_POINT_LOAD, nn * ((c.s + 2) * rt + c.npairs * ct), st);
                launch_pointwise_load<T, T>(c, in, b0_of<T>(c),
                                            op == FCRKPM_OP_FR ? vol_of<T>(c) : nullptr, P, st);
            }
            conv_many_to_one<T>(c, c.prog_bwd, P, U, st);
            ProfScope ps(c, KD_UNPACK, nn * (ct + 1 + rt), st);
            launch_unpack_re<T, T>(U, c.chi, out, c.nn, st);
            break;
        }
        case FCRKPM_OP_UH:
        case FCRKPM_OP_VN: {
            {
                ProfScope ps(c, KD_PACK, nn * (rt + 1 + ct), st);
                launch_pack<T, T>(in, c.chi, U, c.nn, st);
            }
            conv_one_to_many<T>(c, c.prog_fwd, U, P, st);
            ProfScope ps(c, KD_POINT_UH, nn * (c.npairs * ct + (c.s + 2) * rt), st);
            launch_pointwise_uh<T, T>(c, P, b0_of<T>(c), op == FCRKPM_OP_VN ? vol_of<T>(c) : nullptr,
                                      out, st);
            break;
        }
        default:
            fail(FCRKPM_ERR_ARG, "unknown operator");
    }
}

// ---------------------------------------------------------------- solvers

enum { V_B = 0, V_X = 1, V_R = 2, V_P = 3, V_Q = 4, V_T = 5 };
enum { S_RR0 = 0, S_RR1 = 1, S_BREAK = 3, S_NORM = 4, S_BB = 5 };

double read_scalar(Ctx& c, int idx, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(c.hscal, c.scal + idx, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return c.hscal[0];
}

template <typename T>
double dot_to(Ctx& c, const T* a, const T* b, int idx, hipStream_t st)
{
    launch_dot_partial<T>(a, b, c.nn, c.partial, st);
    launch_reduce_to(c.partial, c.scal + idx, st);
    return read_scalar(c, idx, st);
}

struct CgResult {
    int iters = 0;
    double relres = 0.0;
    bool breakdown = false;
    bool converged = false;
};

// CG on chi_Omega K chi_Omega from x with residual r (both in/out), for
// ||r|| / sqrt(bb) <= tol.  p, q: scratch.  Convergence is read every
// `check` iterations.
template <typename T>
CgResult cg_run(Ctx& c, T* x, T* r, T* p, T* q, double bb, double tol, int maxit, int& matvecs,
                hipStream_t st)
{
    CgResult res;
    const double bn = sqrt(bb > 0.0 ? bb : 1.0);
    HIPCHK(hipMemcpyAsync(p, r, sizeof(T) * c.nn, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(c.scal + S_BREAK, 0, sizeof(double), st));
    launch_dot_partial<T>(r, r, c.nn, c.partial, st);
    launch_reduce_to(c.partial, c.scal + S_RR0, st);
    double rr = read_scalar(c, S_RR0, st);
    int parity = 0;
    res.relres = sqrt(rr) / bn;
    if (res.relres <= tol) {
        res.converged = true;
        return res;
    }
    double* pq_part = c.partial;
    double* rr_part = c.partial + kRedBlocks;
    const int check = 4;
    int it = 0;
    while (it < maxit) {
        apply_one<T>(c, FCRKPM_OP_K, p, q, st);
        ++matvecs;
        launch_dot_partial<T>(p, q, c.nn, pq_part, st);
        launch_cg_xr<T>(x, r, p, q, c.nn, pq_part, c.scal, parity, rr_part, st);
        launch_cg_p<T>(p, r, c.nn, rr_part, c.scal, parity, st);
        parity ^= 1;
        ++it;
        if (it % check == 0 || it == maxit) {
            HIPCHK(hipMemcpyAsync(c.hscal, c.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            rr = c.hscal[parity];
            res.relres = sqrt(rr) / bn;
            if (c.hscal[S_BREAK] != 0.0) {
                res.breakdown = true;
                break;
            }
            if (res.relres <= tol) {
                res.converged = true;
                break;
            }
        }
    }
    res.iters = it;
    return res;
}

// Solve chi_Omega K chi_Omega x = b with b in v64[V_B] and the initial x in
// v64[V_X] (zero off the free nodes).  Returns status; fills info.
fcrkpm_status solve_core(Ctx& c, int mode, double tol, int maxit, fcrkpm_info* info,
                         hipStream_t st)
{
    const long nn = c.nn;
    double* b = c.v64 + V_B * nn;
    double* x = c.v64 + V_X * nn;
    double* r = c.v64 + V_R * nn;
    double* p = c.v64 + V_P * nn;
    double* q = c.v64 + V_Q * nn;
    fcrkpm_info inf;
    memset(&inf, 0, sizeof(inf));
    const double bb = dot_to<double>(c, b, b, S_BB, st);
    fcrkpm_status status = FCRKPM_OK;
    if (bb == 0.0) {
        HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * nn, st));
        inf.rel_res = 0.0;
        inf.true_rel_res = 0.0;
        if (info) *info = inf;
        return FCRKPM_OK;
    }
    const double bn = sqrt(bb);
    int total = 0;
    bool need_f64 = (mode == FCRKPM_MODE_F64);
    if (mode == FCRKPM_MODE_F32_REFINED) {
        float* x32 = c.v32 + 0 * nn;
        float* r32 = c.v32 + 1 * nn;
        float* p32 = c.v32 + 2 * nn;
        float* q32 = c.v32 + 3 * nn;
        double prev = INFINITY;
        for (int outer = 0; outer < 60; ++outer) {
            apply_one<double>(c, FCRKPM_OP_K, x, q, st);
            ++inf.matvecs_f64;
            launch_sub_masked(b, q, c.freem, r, nn, st);
            const double rr = dot_to<double>(c, r, r, S_NORM, st);
            const double rel = sqrt(rr) / bn;
            inf.rel_res = rel;
            if (rel <= tol) break;
            if (total >= maxit) {
                status = FCRKPM_ERR_NOCONV;
                break;
            }
            if (!(rel < 0.5 * prev)) {  // refinement stagnates: finish in FP64
                need_f64 = true;
                inf.fallback_used = 1;
                break;
            }
            prev = rel;
            ++inf.outer_iters;
            launch_scale_to32(r, c.scal, S_NORM, r32, nn, st);
            HIPCHK(hipMemsetAsync(x32, 0, sizeof(float) * nn, st));
            double itol = 0.5 * tol / rel;
            itol = std::min(0.1, std::max(itol, 2e-6));
            CgResult cr = cg_run<float>(c, x32, r32, p32, q32, 1.0, itol, maxit - total,
                                        inf.matvecs_f32, st);
            total += cr.iters;
            launch_axpy32to64(x, x32, c.scal, S_NORM, nn, st);
        }
    }
    if (need_f64) {
        apply_one<double>(c, FCRKPM_OP_K, x, q, st);
        ++inf.matvecs_f64;
        launch_sub_masked(b, q, c.freem, r, nn, st);
        CgResult cr = cg_run<double>(c, x, r, p, q, bb, tol, std::max(1, maxit - total),
                                     inf.matvecs_f64, st);
        total += cr.iters;
        inf.rel_res = cr.relres;
        if (cr.breakdown || !cr.converged) status = FCRKPM_ERR_NOCONV;
    }
    inf.iters = total;
    // true residual in FP64
    apply_one<double>(c, FCRKPM_OP_K, x, q, st);
    launch_sub_masked(b, q, c.freem, r, nn, st);
    inf.true_rel_res = sqrt(dot_to<double>(c, r, r, S_NORM, st)) / bn;
    if (mode == FCRKPM_MODE_F32_REFINED && !need_f64 && inf.rel_res > tol) status = FCRKPM_ERR_NOCONV;
    if (info) *info = inf;
    return status;
}

}  // namespace

// ========================================================================= ABI

namespace {
fcrkpm_status run_guarded(std::string& err, const std::function<fcrkpm_status()>& body)
{
    try {
        fcrkpm_status s = body();
        if (s == FCRKPM_OK) err.clear();
        return s;
    } catch (const ArgFail& a) {
        err = a.msg;
        return a.st;
    } catch (const HipFail& h) {
        err = std::string("HIP error ") + hipGetErrorString(h.e) + " in " + h.what;
        return FCRKPM_ERR_HIP;
    } catch (const std::bad_alloc&) {
        err = "host allocation failed";
        return FCRKPM_ERR_OOM;
    } catch (...) {
        err = "unexpected exception";
        return FCRKPM_ERR_HIP;
    }
}
}  // namespace

extern "C" fcrkpm_status fcrkpm_setup(const fcrkpm_grid* grid, const uint8_t* mask, int32_t kernel,
                                      const double support[3], int32_t degree, void* stream,
                                      fcrkpm_ctx** out)
{
    if (out) *out = nullptr;
    fcrkpm_ctx* h = nullptr;
    fcrkpm_status s = run_guarded(g_setup_err, [&]() -> fcrkpm_status {
        if (!grid || !mask || !support || !out) fail(FCRKPM_ERR_ARG, "NULL argument");
        if (kernel != FCRKPM_KERNEL_CUBIC_BSPLINE) fail(FCRKPM_ERR_ARG, "unknown kernel");
        if (grid->dim < 1 || grid->dim > 3) fail(FCRKPM_ERR_ARG, "dim must be 1, 2 or 3");
        if (degree < 1 || degree > 2) fail(FCRKPM_ERR_ARG, "degree must be 1 or 2");
        if (grid->flags != 0) fail(FCRKPM_ERR_ARG, "flags must be 0");
        hipStream_t st = (hipStream_t)stream;
        h = new fcrkpm_ctx();
        Ctx& c = h->c;
        c.dim = grid->dim;
        c.degree = degree;
        for (int a = 0; a < 3; ++a) {
            c.n[a] = grid->n[a];
            if (a < c.dim) {
                if (c.n[a] < 4 || c.n[a] > 1024) fail(FCRKPM_ERR_ARG, "box size per axis must be in [4, 1024]");
                if (!(grid->h[a] > 0.0) || !isfinite(grid->h[a])) fail(FCRKPM_ERR_ARG, "spacing must be positive");
                if (!(support[a] >= 1.0) || !isfinite(support[a])) fail(FCRKPM_ERR_ARG, "support must be >= 1");
                c.h[a] = grid->h[a];
                c.at[a] = support[a];
                c.m[a] = (int)floor(support[a]);
                if (2 * c.m[a] >= c.n[a]) fail(FCRKPM_ERR_ARG, "support too large for the box");
                if (!make_plan(c.n[a], c.plan[a])) fail(FCRKPM_ERR_ARG, "box size must factor into 2, 3 and 5");
            } else {
                if (c.n[a] != 1) fail(FCRKPM_ERR_ARG, "unused axes must have n = 1");
                c.h[a] = 1.0;
                c.at[a] = 0.0;
                c.m[a] = 0;
                c.plan[a].n = 1;
                c.plan[a].nst = 0;
            }
        }
        c.nn = (long)c.n[0] * c.n[1] * c.n[2];
        int exs[kMaxS][3];
        c.s = monomials(c.dim, degree, exs, kMaxS);
        memcpy(c.ex, exs, sizeof(exs));
        int ex2[kMaxMono][3];
        c.nmono2 = monomials(c.dim, 2 * degree, ex2, kMaxMono);
        memcpy(c.ex2, ex2, sizeof(ex2));
        c.naxes = 0;
        for (int a = 0; a < c.dim; ++a) c.axes[c.naxes++] = a;
        const long nn = c.nn;

        // masks and volumes
        c.chi = dalloc<uint8_t>(nn);
        c.freem = dalloc<uint8_t>(nn);
        c.dirm = dalloc<uint8_t>(nn);
        c.dflag = dalloc<int>(8);
        HIPCHK(hipMemcpyAsync(c.chi, mask, nn, hipMemcpyDeviceToDevice, st));
        if (grid->dirichlet)
            HIPCHK(hipMemcpyAsync(c.dirm, grid->dirichlet, nn, hipMemcpyDeviceToDevice, st));
        else
            HIPCHK(hipMemsetAsync(c.dirm, 0, nn, st));
        int init[8] = {0x7fffffff, 0x7fffffff, 0, 0, 0, 0, 0, 0};
        HIPCHK(hipMemcpyAsync(c.dflag, init, sizeof(init), hipMemcpyHostToDevice, st));
        launch_free_mask(c.chi, c.dirm, c.freem, c.dflag + 0, nn, st);
        c.vol64 = dalloc<double>(nn);
        c.vol32 = dalloc<float>(nn);
        launch_vol(c.chi, grid->vol, c.h[0] * c.h[1] * c.h[2], c.vol64, c.vol32, nn, st);
        // periodic-gap check on each axis (Sec 5.1, Eq 66)
        int ntot = c.n[0] + c.n[1] + c.n[2];
        int* occ = dalloc<int>(ntot);
        HIPCHK(hipMemsetAsync(occ, 0, sizeof(int) * ntot, st));
        launch_axis_extent(c, c.chi, occ, st);
        std::vector<int> hocc(ntot);
        int hflag[8];
        HIPCHK(hipMemcpyAsync(hocc.data(), occ, sizeof(int) * ntot, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hflag, c.dflag, sizeof(hflag), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        dfree(occ);
        if (hflag[0] != 0x7fffffff)
            fail(FCRKPM_ERR_ARG, "Dirichlet node " + std::to_string(hflag[0]) + " lies outside the domain mask");
        int off = 0;
        for (int a = 0; a < 3; ++a) {
            int lo = -1, hi = -1;
            for (int i = 0; i < c.n[a]; ++i)
                if (hocc[off + i]) {
                    if (lo < 0) lo = i;
                    hi = i;
                }
            if (lo < 0) fail(FCRKPM_ERR_ARG, "empty domain mask");
            bool full = true;  // a domain filling the axis is periodic along it
            for (int i = 0; i < c.n[a]; ++i) full = full && hocc[off + i];
            if (a < c.dim && !full && hi - lo > c.n[a] - c.m[a] - 1)
                fail(FCRKPM_ERR_ARG, "domain extent on axis " + std::to_string(a) +
                                         " leaves a periodic gap below floor(support)+1 nodes");
            off += c.n[a];
        }

        // twiddles and separable kernel spectra (Sec 5.2-5.3, Eq 68-79)
        const long double twopi = 6.283185307179586476925286766559005768L;
        for (int a = 0; a < 3; ++a) {
            int L = c.n[a];
            std::vector<cplx<double>> tw(L);
            std::vector<cplx<float>> twf(L);
            for (int k = 0; k < L; ++k) {
                long double ang = twopi * (long double)k / (long double)L;
                tw[k] = {(double)cosl(ang), (double)(-sinl(ang))};
                twf[k] = {(float)tw[k].x, (float)tw[k].y};
            }
            c.tw64[a] = dalloc<cplx<double>>(L);
            c.tw32[a] = dalloc<cplx<float>>(L);
            HIPCHK(hipMemcpyAsync(c.tw64[a], tw.data(), sizeof(cplx<double>) * L, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(c.tw32[a], twf.data(), sizeof(cplx<float>) * L, hipMemcpyHostToDevice, st));
            int ne = (a < c.dim) ? 2 * degree + 1 : 1;
            std::vector<cplx<double>> sp((size_t)ne * L);
            std::vector<cplx<float>> spf((size_t)ne * L);
            for (int e = 0; e < ne; ++e)
                for (int k = 0; k < L; ++k) {
                    long double re = 0.0L, im = 0.0L;
                    if (a < c.dim) {
                        for (int o = -c.m[a]; o <= c.m[a]; ++o) {
                            long double w = bspline((long double)o / (long double)c.at[a]);
                            long double mo = 1.0L;
                            for (int t = 0; t < e; ++t) mo *= (long double)o;
                            long double ang = twopi * (long double)((long)k * o % L) / (long double)L;
                            re += mo * w * cosl(ang);
                            im -= mo * w * sinl(ang);
                        }
                    } else {
                        re = 1.0L;
                    }
                    sp[(size_t)e * L + k] = {(double)re, (double)im};
                    spf[(size_t)e * L + k] = {(float)re, (float)im};
                }
            c.spec64[a] = dalloc<cplx<double>>(sp.size());
            c.spec32[a] = dalloc<cplx<float>>(spf.size());
            HIPCHK(hipMemcpyAsync(c.spec64[a], sp.data(), sizeof(cplx<double>) * sp.size(), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(c.spec32[a], spf.data(), sizeof(cplx<float>) * spf.size(), hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        build_prog_fwd(c, c.prog_fwd);
        build_prog_bwd(c, c.prog_bwd);
        ConvProg prog_mom;
        build_prog_mom(c, prog_mom);

        // Alg 1: moment convolutions and per-node solves (FP64)
        c.b0_64 = dalloc<double>((size_t)c.s * nn);
        c.ba_64 = dalloc<double>((size_t)c.dim * c.s * nn);
        c.b0_32 = dalloc<float>((size_t)c.s * nn);
        c.ba_32 = dalloc<float>((size_t)c.dim * c.s * nn);
        {
            int npm = prog_mom.nio;
            cplx<double>* G = dalloc<cplx<double>>((size_t)(npm + 1) * nn);
            cplx<double>* U = G + (size_t)npm * nn;
            launch_chi_pack(c.chi, U, nn, st);
            conv_one_to_many<double>(c, prog_mom, U, G, st);
            launch_moment_solve(c, G, c.dflag + 1, st);
            HIPCHK(hipMemcpyAsync(hflag, c.dflag, sizeof(hflag), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            dfree(G);
            if (hflag[1] != 0x7fffffff)
                fail(FCRKPM_ERR_SINGULAR, "moment matrix not positive definite at node " + std::to_string(hflag[1]));
        }

        // workspace
        c.npairs = (c.s + 1) / 2;
        c.work64 = dalloc<cplx<double>>((size_t)(c.npairs + 1) * nn);
        c.work32 = dalloc<cplx<float>>((size_t)(c.npairs + 1) * nn);
        c.v64 = dalloc<double>((size_t)6 * nn);
        c.v32 = dalloc<float>((size_t)5 * nn);
        c.partial = dalloc<double>(2 * kRedBlocks);
        c.scal = dalloc<double>(16);
        HIPCHK(hipMemsetAsync(c.scal, 0, 16 * sizeof(double), st));
        HIPCHK(hipHostMalloc((void**)&c.hscal, 16 * sizeof(double), hipHostMallocDefault));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        *out = h;
        h = nullptr;
        return FCRKPM_OK;
    });
    if (h) {
        release(h->c);
        delete h;
    }
    return s;
}

extern "C" fcrkpm_status fcrkpm_apply(fcrkpm_ctx* ctx, int32_t op, int32_t dtype, int32_t nrhs,
                                      const void* in, void* out, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (op < FCRKPM_OP_K || op > FCRKPM_OP_VN) fail(FCRKPM_ERR_ARG, "unknown operator");
        if (dtype != FCRKPM_F64 && dtype != FCRKPM_F32) fail(FCRKPM_ERR_ARG, "unknown dtype");
        if (nrhs < 1) fail(FCRKPM_ERR_ARG, "nrhs must be >= 1");
        if (!in || !out) fail(FCRKPM_ERR_ARG, "NULL array");
        const size_t es = dtype == FCRKPM_F64 ? 8 : 4;
        const char* a0 = (const char*)in;
        const char* b0 = (const char*)out;
        const size_t bytes = es * (size_t)c.nn * nrhs;
        if (a0 < b0 + bytes && b0 < a0 + bytes) fail(FCRKPM_ERR_ARG, "in and out overlap");
        hipStream_t st = (hipStream_t)stream;
        for (int j = 0; j < nrhs; ++j) {
            if (dtype == FCRKPM_F64)
                apply_one<double>(c, op, (const double*)in + (size_t)j * c.nn, (double*)out + (size_t)j * c.nn, st);
            else
                apply_one<float>(c, op, (const float*)in + (size_t)j * c.nn, (float*)out + (size_t)j * c.nn, st);
        }
        HIPCHK(hipGetLastError());
        return FCRKPM_OK;
    });
}

extern "C" fcrkpm_status fcrkpm_solve(fcrkpm_ctx* ctx, int32_t mode, int32_t nrhs, const double* r,
                                      const double* g, double* d_inout, double* uh_out, double tol,
                                      int32_t maxit, fcrkpm_info* info, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (mode != FCRKPM_MODE_F64 && mode != FCRKPM_MODE_F32_REFINED) fail(FCRKPM_ERR_ARG, "unknown mode");
        if (nrhs < 1 || !r || !d_inout) fail(FCRKPM_ERR_ARG, "bad arguments");
        if (!(tol > 0.0) || maxit < 1) fail(FCRKPM_ERR_ARG, "tol must be > 0 and maxit >= 1");
        hipStream_t st = (hipStream_t)stream;
        const long nn = c.nn;
        fcrkpm_status worst = FCRKPM_OK;
        for (int j = 0; j < nrhs; ++j) {
            const double* rj = r + (size_t)j * nn;
            const double* gj = g ? g + (size_t)j * nn : nullptr;
            double* dj = d_inout + (size_t)j * nn;
            HIPCHK(hipMemsetAsync(c.dflag + 2, 0, sizeof(int), st));
            launch_check_finite(rj, nn, c.dflag + 2, st);
            if (gj) launch_check_finite(gj, nn, c.dflag + 2, st);
            int hf = 0;
            HIPCHK(hipMemcpyAsync(&hf, c.dflag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (hf) fail(FCRKPM_ERR_ARG, "non-finite value in r or g");
            double* b = c.v64 + V_B * nn;
            double* x = c.v64 + V_X * nn;
            double* t = c.v64 + V_T * nn;
            double* p = c.v64 + V_P * nn;
            double* q = c.v64 + V_Q * nn;
            apply_one<double>(c, FCRKPM_OP_FR, rj, t, st);  // f^r (Alg 4)
            if (gj) {
                launch_masked_copy<double>(gj, c.dirm, p, nn, st);  // d_Gamma
                apply_one<double>(c, FCRKPM_OP_K_FULL, p, q, st);
                launch_sub_masked(t, q, c.freem, b, nn, st);
            } else {
                launch_masked_copy<double>(t, c.freem, b, nn, st);
            }
            launch_masked_copy<double>(dj, c.freem, x, nn, st);
            fcrkpm_info inf;
            fcrkpm_status s = solve_core(c, mode, tol, maxit, &inf, st);
            if (s != FCRKPM_OK) worst = s;
            if (gj) {
                launch_masked_copy<double>(gj, c.dirm, p, nn, st);
                launch_select(c.freem, x, p, dj, nn, st);
            } else {
                HIPCHK(hipMemcpyAsync(dj, x, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
            }
            if (uh_out) apply_one<double>(c, FCRKPM_OP_UH, dj, uh_out + (size_t)j * nn, st);
            if (info) *info = inf;
        }
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (worst != FCRKPM_OK) c.err = "solver did not reach the tolerance";
        return worst;
    });
}

extern "C" fcrkpm_status fcrkpm_adjoint(fcrkpm_ctx* ctx, int32_t mode, int32_t nrhs,
                                        const double* dl_duh, double* dl_dr, double tol,
                                        int32_t maxit, fcrkpm_info* info, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (mode != FCRKPM_MODE_F64 && mode != FCRKPM_MODE_F32_REFINED) fail(FCRKPM_ERR_ARG, "unknown mode");
        if (nrhs < 1 || !dl_duh || !dl_dr) fail(FCRKPM_ERR_ARG, "bad arguments");
        if (!(tol > 0.0) || maxit < 1) fail(FCRKPM_ERR_ARG, "tol must be > 0 and maxit >= 1");
        hipStream_t st = (hipStream_t)stream;
        const long nn = c.nn;
        fcrkpm_status worst = FCRKPM_OK;
        for (int j = 0; j < nrhs; ++j) {
            double* b = c.v64 + V_B * nn;
            double* x = c.v64 + V_X * nn;
            double* t = c.v64 + V_T * nn;
            apply_one<double>(c, FCRKPM_OP_NT, dl_duh + (size_t)j * nn, t, st);
            launch_masked_copy<double>(t, c.freem, b, nn, st);
            HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * nn, st));
            fcrkpm_info inf;
            fcrkpm_status s = solve_core(c, mode, tol, maxit, &inf, st);
            if (s != FCRKPM_OK) worst = s;
            apply_one<double>(c, FCRKPM_OP_VN, x, dl_dr + (size_t)j * nn, st);
            if (info) *info = inf;
        }
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (worst != FCRKPM_OK) c.err = "adjoint solve did not reach the tolerance";
        return worst;
    });
}

extern "C" fcrkpm_status fcrkpm_get_coeffs(fcrkpm_ctx* ctx, int32_t which, double* out, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (!out) fail(FCRKPM_ERR_ARG, "NULL array");
        hipStream_t st = (hipStream_t)stream;
        switch (which) {
            case FCRKPM_COEF_B0:
                HIPCHK(hipMemcpyAsync(out, c.b0_64, sizeof(double) * c.s * c.nn, hipMemcpyDeviceToDevice, st));
                break;
            case FCRKPM_COEF_BALPHA:
                HIPCHK(hipMemcpyAsync(out, c.ba_64, sizeof(double) * c.dim * c.s * c.nn, hipMemcpyDeviceToDevice, st));
                break;
            case FCRKPM_COEF_FREE:
                launch_mask_to_double(c.freem, out, c.nn, st);
                break;
            default:
                fail(FCRKPM_ERR_ARG, "unknown coefficient field");
        }
        HIPCHK(hipGetLastError());
        return FCRKPM_OK;
    });
}


extern "C" fcrkpm_status fcrkpm_profile(fcrkpm_ctx* ctx, int32_t enable)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (!c.prof) {
            Prof* p = new Prof();
            c.prof = p;
            for (auto& k : p->k)
                for (auto& e : k.ev) HIPCHK(hipEventCreate(&e));
        }
        Prof* p = (Prof*)c.prof;
        if (enable) {  // a new sampling window; disabling keeps the samples readable
            HIPCHK(hipDeviceSynchronize());
            for (auto& k : p->k) {
                k.launches = 0;
                k.bytes = 0.0;
                k.nrec = 0;
            }
        }
        c.prof_on = enable != 0;
        return FCRKPM_OK;
    });
}

extern "C" fcrkpm_status fcrkpm_profile_read(fcrkpm_ctx* ctx, int32_t kind, int64_t* launches,
                                             double* mean_ms, double* bytes_per_launch)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (kind < 0 || kind >= KD_NKINDS) fail(FCRKPM_ERR_ARG, "unknown kernel kind");
        if (!c.prof) fail(FCRKPM_ERR_ARG, "profiling was never enabled");
        Prof* p = (Prof*)c.prof;
        ProfKind& k = p->k[kind];
        HIPCHK(hipDeviceSynchronize());
        double tot = 0.0;
        for (int i = 0; i < k.nrec; ++i) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, k.ev[2 * i], k.ev[2 * i + 1]));
            tot += ms;
        }
        if (launches) *launches = k.launches;
        if (mean_ms) *mean_ms = k.nrec ? tot / k.nrec : 0.0;
        if (bytes_per_launch) *bytes_per_launch = k.launches ? k.bytes / (double)k.launches : 0.0;
        return FCRKPM_OK;
    });
}

extern "C" int32_t fcrkpm_kernel_kinds(void) { return KD_NKINDS; }

extern "C" const char* fcrkpm_kernel_name(int32_t kind)
{
    return (kind >= 0 && kind < KD_NKINDS) ? kKindNames[kind] : "";
}

extern "C" int32_t fcrkpm_basis_size(const fcrkpm_ctx* ctx) { return ctx ? ctx->c.s : -1; }

extern "C" void fcrkpm_destroy(fcrkpm_ctx* ctx)
{
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    release(ctx->c);
    delete ctx;
}

extern "C" const char* fcrkpm_last_error(const fcrkpm_ctx* ctx)
{
    return ctx ? ctx->c.err.c_str() : g_setup_err.c_str();
}

extern "C" const char* fcrkpm_status_str(fcrkpm_status s)
{
    switch (s) {
        case FCRKPM_OK: return "FCRKPM_OK";
        case FCRKPM_ERR_ARG: return "FCRKPM_ERR_ARG";
        case FCRKPM_ERR_SINGULAR: return "FCRKPM_ERR_SINGULAR";
        case FCRKPM_ERR_NOCONV: return "FCRKPM_ERR_NOCONV";
        case FCRKPM_ERR_HIP: return "FCRKPM_ERR_HIP";
        case FCRKPM_ERR_OOM: return "FCRKPM_ERR_OOM";
        case FCRKPM_ERR_UNSUPPORTED: return "FCRKPM_ERR_UNSUPPORTED";
    }
    return "FCRKPM_ERR_UNKNOWN";
}

extern "C" int32_t fcrkpm_version(void) { return 100; }
