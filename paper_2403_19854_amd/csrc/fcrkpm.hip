// fcrkpm.hip -- host side of the C ABI declared in include/fcrkpm.h: argument
// checks, plans and spectral tables, the convolution pipelines of Alg 1-4,
// the CG drivers (FP64, and FP32 inside FP64 iterative refinement) and the
// adjoint solve.
#include <hip/hip_runtime.h>

#include <math.h>
#include <cmath>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <type_traits>
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
    KD_P1_X, KD_P1_Y, KD_P1_Z, KD_MID_K, KD_MID_UH, KD_MID_LOAD, KD_P2_X, KD_P2_Y, KD_P2_Z,
    KD_SETUP_PASS, KD_STAGES
};
constexpr int KD_NKINDS = 2 * KD_STAGES;  // FP64 kinds, then FP32 kinds
const char* const kStageNames[KD_STAGES] = {
    "sep_part1_x", "sep_part1_y", "sep_part1_z", "sep_mid_k", "sep_mid_uh", "sep_mid_load",
    "sep_part2_x", "sep_part2_y", "sep_part2_z", "sep_setup_pass"};
std::string kind_name(int k)
{
    return std::string(kStageNames[k % KD_STAGES]) + (k >= KD_STAGES ? "_f32" : "_f64");
}
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
    dfree(c.dprog);
    if (c.hscal) (void)hipHostFree(c.hscal);
    c.hscal = nullptr;
    for (auto& e : c.poll_ev)
        if (e) (void)hipEventDestroy(e);
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

// Programs of the separable passes for a monomial list (basis order for
// Alg 2-4, degree <= 2n for Alg 1).  P_j lists the distinct exponent prefixes
// over the first j+1 active axes; P_{k-1} is the list itself.  Part 1 maps
// P_{j-1} -> P_j with kernel t_e (Eq 77), part 2 maps P_j -> P_{j-1} with the
// reflected kernel (-1)^e t_e (Eq 55, 78).  Coefficients carry the 1/2 of the
// pair separation and the 1/L of each inverse transform.
SepPlan build_plan(const Ctx& c, const int (*mono)[3], int nm)
{
    SepPlan sp;
    sp.k = c.naxes;
    const int k = sp.k;
    std::vector<std::vector<std::vector<int>>> P(k);
    for (int j = 0; j < k; ++j) {
        for (int m = 0; m < nm; ++m) {
            std::vector<int> tup;
            for (int q = 0; q <= j; ++q) tup.push_back(mono[m][c.axes[q]]);
            if (j == k - 1 || std::find(P[j].begin(), P[j].end(), tup) == P[j].end())
                P[j].push_back(tup);
        }
        sp.size[j] = (int)P[j].size();
        if ((int)P[j].size() > kMaxSepOut) fail(FCRKPM_ERR_UNSUPPORTED, "too many monomials");
    }
    auto index_of = [&](int j, const std::vector<int>& tup) {
        if (j < 0) return 0;
        return (int)(std::find(P[j].begin(), P[j].end(), tup) - P[j].begin());
    };
    for (int j = 0; j < k; ++j) {
        const double inv = 1.0 / (2.0 * c.n[c.axes[j]]);
        SepProg& f = sp.p1[j];
        memset(&f, 0, sizeof(f));
        f.nin = (j == 0) ? 1 : sp.size[j - 1];
        f.nout = sp.size[j];
        int t = 0;
        for (int o = 0; o < f.nout; ++o) {
            f.ostart[o] = t;
            std::vector<int> pre(P[j][o].begin(), P[j][o].end() - 1);
            f.t[t++] = SepTerm{o, index_of(j - 1, pre), P[j][o].back(), 0, inv};
        }
        f.ostart[f.nout] = t;
        SepProg& g = sp.p2[j];
        memset(&g, 0, sizeof(g));
        g.nin = sp.size[j];
        g.nout = (j == 0) ? 1 : sp.size[j - 1];
        t = 0;
        for (int o = 0; o < g.nout; ++o) {
            g.ostart[o] = t;
            for (int i = 0; i < g.nin; ++i) {
                std::vector<int> pre(P[j][i].begin(), P[j][i].end() - 1);
                if (index_of(j - 1, pre) != o) continue;
                const int e = P[j][i].back();
                if (t >= kMaxSepTerms) fail(FCRKPM_ERR_UNSUPPORTED, "too many terms");
                g.t[t++] = SepTerm{o, i, e, 0, (e & 1) ? -inv : inv};
            }
        }
        g.ostart[g.nout] = t;
    }
    sp.maxpairs = 1;
    for (int j = 0; j + 1 < k; ++j) sp.maxpairs = std::max(sp.maxpairs, (sp.size[j] + 1) / 2);
    return sp;
}

template <typename T>
cplx<T>* work_of(Ctx& c)
{
    if constexpr (sizeof(T) == 8) return c.work64;
    else return c.work32;
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

template <typename T>
int kind_of(int stage) { return stage + (sizeof(T) == 4 ? KD_STAGES : 0); }

// bytes of `nreal` real fields stored as complex pairs
template <typename T>
double pair_bytes(int nreal) { return (double)((nreal + 1) / 2) * sizeof(cplx<T>); }

// Part-1 passes on axes 0..k-2 (Alg 2/3 first half): the field `in` (Tio,
// masked) becomes P_{k-2} pairs; returns the slot that holds them.
template <typename T, typename Tio>
cplx<T>* part1(Ctx& c, const SepPlan& sp, const Tio* in, const uint8_t* mask, cplx<T>* S1,
               cplx<T>* S2, hipStream_t st)
{
    const double nn = (double)c.nn;
    const void* src = in;
    cplx<T>* dst = S1;
    for (int j = 0; j + 1 < sp.k; ++j) {
        const int ldm = (j == 0) ? SEP_LD_REAL : SEP_LD_PAIRS;
        const double inb = (j == 0) ? sizeof(Tio) + 1.0 : pair_bytes<T>(sp.size[j - 1]);
        ProfScope ps(c, kind_of<T>(KD_P1_X + c.axes[j]), nn * (inb + pair_bytes<T>(sp.size[j])), st);
        launch_sep_pass<T, Tio>(c, c.axes[j], sp.p1[j], sp.d1[j], ldm, src, mask, SEP_ST_PAIRS, dst, nullptr,
                                nullptr, nullptr, st);
        src = dst;
        dst = (dst == S1) ? S2 : S1;
    }
    return (cplx<T>*)src;
}

// Part-2 passes on axes k-2..0 from P_{k-2} pairs in `cur` to the real field
// `out` (masked).
template <typename T, typename Tio>
void part2(Ctx& c, const SepPlan& sp, cplx<T>* cur, cplx<T>* S1, cplx<T>* S2, Tio* out,
           const uint8_t* mask, hipStream_t st)
{
    const double nn = (double)c.nn;
    for (int j = sp.k - 2; j >= 0; --j) {
        const double inb = pair_bytes<T>(sp.size[j]);
        if (j > 0) {
            cplx<T>* dst = (cur == S1) ? S2 : S1;
            ProfScope ps(c, kind_of<T>(KD_P2_X + c.axes[j]), nn * (inb + pair_bytes<T>(sp.size[j - 1])), st);
            launch_sep_pass<T, Tio>(c, c.axes[j], sp.p2[j], sp.d2[j], SEP_LD_PAIRS, cur, nullptr, SEP_ST_PAIRS,
                                    dst, nullptr, nullptr, nullptr, st);
            cur = dst;
        } else {
            ProfScope ps(c, kind_of<T>(KD_P2_X + c.axes[j]), nn * (inb + sizeof(Tio) + 1.0), st);
            launch_sep_pass<T, Tio>(c, c.axes[j], sp.p2[j], sp.d2[j], SEP_LD_PAIRS, cur, nullptr, SEP_ST_REAL,
                                    out, mask, nullptr, nullptr, st);
        }
    }
}

// One operator on one field, arithmetic precision T, field type Tio (Alg 2, 3, 4).
template <typename T, typename Tio = T>
void apply_one(Ctx& c, int op, const Tio* in, Tio* out, hipStream_t st)
{
    const SepPlan& sp = c.basis_plan;
    const int k = sp.k, last = c.axes[k - 1];
    cplx<T>* S1 = work_of<T>(c);
    cplx<T>* S2 = S1 + (size_t)sp.maxpairs * c.nn;
    const double nn = (double)c.nn, rt = sizeof(T);
    const double inb1 = (k == 1) ? sizeof(Tio) + 1.0 : pair_bytes<T>(k >= 2 ? sp.size[k - 2] : 1);
    const double outb2 = (k == 1) ? sizeof(Tio) + 1.0 : pair_bytes<T>(k >= 2 ? sp.size[k - 2] : 1);
    switch (op) {
        case FCRKPM_OP_K:
        case FCRKPM_OP_K_FULL: {
            const uint8_t* mk = (op == FCRKPM_OP_K) ? c.freem : c.chi;
            cplx<T>* cur = part1<T, Tio>(c, sp, in, mk, S1, S2, st);
            cplx<T>* dst = (cur == S1) ? S2 : S1;
            {
                ProfScope ps(c, kind_of<T>(KD_MID_K), nn * (inb1 + outb2 + (c.dim * c.s + 1) * rt), st);
                if (k == 1)
                    launch_sep_mid<T, Tio>(c, last, sp.p1[0], sp.d1[0], sp.p2[0], sp.d2[0], SEP_PW_K, SEP_LD_REAL, in, mk,
                                           SEP_ST_REAL, out, mk, nullptr, b0_of<T>(c), ba_of<T>(c),
                                           vol_of<T>(c), nullptr, nullptr, st);
                else
                    launch_sep_mid<T, Tio>(c, last, sp.p1[k - 1], sp.d1[k - 1], sp.p2[k - 1], sp.d2[k - 1], SEP_PW_K, SEP_LD_PAIRS,
                                           cur, nullptr, SEP_ST_PAIRS, dst, nullptr, nullptr,
                                           b0_of<T>(c), ba_of<T>(c), vol_of<T>(c), nullptr, nullptr,
                                           st);
            }
            if (k > 1) part2<T, Tio>(c, sp, dst, S1, S2, out, mk, st);
            break;
        }
        case FCRKPM_OP_FR:
        case FCRKPM_OP_NT:
        case FCRKPM_OP_UH:
        case FCRKPM_OP_VN:
            if constexpr (!std::is_same_v<T, Tio>) {
                fail(FCRKPM_ERR_ARG, "mixed precisions are supported for K only");
            } else {
                const T* vol = (op == FCRKPM_OP_FR || op == FCRKPM_OP_VN) ? vol_of<T>(c) : nullptr;
                if (op == FCRKPM_OP_FR || op == FCRKPM_OP_NT) {
                    {
                        ProfScope ps(c, kind_of<T>(KD_MID_LOAD), nn * (sizeof(Tio) + (c.s + 1) * rt + outb2), st);
                        launch_sep_mid<T, Tio>(c, last, sp.p1[k - 1], sp.d1[k - 1], sp.p2[k - 1], sp.d2[k - 1], SEP_PW_LOAD,
                                               SEP_LD_PAIRS, nullptr, nullptr,
                                               k == 1 ? SEP_ST_REAL : SEP_ST_PAIRS,
                                               k == 1 ? (void*)out : (void*)S1, c.chi, in,
                                               b0_of<T>(c), ba_of<T>(c), vol, nullptr, nullptr, st);
                    }
                    if (k > 1) part2<T, Tio>(c, sp, S1, S1, S2, out, c.chi, st);
                } else {
                    cplx<T>* cur = part1<T, Tio>(c, sp, in, c.chi, S1, S2, st);
                    ProfScope ps(c, kind_of<T>(KD_MID_UH), nn * (inb1 + (c.s + 1) * rt + sizeof(Tio)), st);
                    launch_sep_mid<T, Tio>(c, last, sp.p1[k - 1], sp.d1[k - 1], sp.p2[k - 1], sp.d2[k - 1], SEP_PW_UH,
                                           k == 1 ? SEP_LD_REAL : SEP_LD_PAIRS,
                                           k == 1 ? (const void*)in : (const void*)cur, c.chi,
                                           SEP_ST_REAL, out, nullptr, nullptr, b0_of<T>(c),
                                           ba_of<T>(c), vol, nullptr, nullptr, st);
                }
            }
            break;
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

// Look-ahead convergence polling: after each batch of CG iterations the
// device scalars are copied to a pinned slot and an event is recorded; the
// host only waits for the PREVIOUS batch, so the queue never drains while
// the host decides.
struct Poller {
    Ctx& c;
    hipStream_t st;
    int slot = 0;      // slot the next post goes to
    int nposted = 0;   // posts since the last full drain
    int parity_of[2] = {0, 0};
    Poller(Ctx& c_, hipStream_t st_) : c(c_), st(st_) {}
    void post(int parity)
    {
        HIPCHK(hipMemcpyAsync(c.hscal + 8 * slot, c.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(c.poll_ev[slot], st));
        parity_of[slot] = parity;
        ++nposted;
        slot ^= 1;
    }
    void read(int s, double& rr, bool& brk)
    {
        HIPCHK(hipEventSynchronize(c.poll_ev[s]));
        rr = c.hscal[8 * s + parity_of[s]];
        brk = c.hscal[8 * s + S_BREAK] != 0.0;
    }
    // scalars of the second-to-last post (the last one may still run); false if none
    bool wait_prev(double& rr, bool& brk)
    {
        if (nposted < 2) return false;
        read(slot, rr, brk);
        return true;
    }
    // scalars of the last post; afterwards nothing is pending
    void wait_last(double& rr, bool& brk)
    {
        read(slot ^ 1, rr, brk);
        nposted = 0;
    }
};

// one CG iteration on vectors of type T with K products in precision TP
template <typename T, typename TP = T>
void cg_iteration(Ctx& c, T* x, T* r, T* p, T* q, int& parity, int& matvecs, hipStream_t st)
{
    double* pq_part = c.partial;
    double* rr_part = c.partial + kRedBlocks;
    apply_one<TP, T>(c, FCRKPM_OP_K, p, q, st);
    ++matvecs;
    launch_dot_partial<T>(p, q, c.nn, pq_part, st);
    launch_cg_xr<T>(x, r, p, q, c.nn, pq_part, c.scal, parity, rr_part, st);
    launch_cg_p<T>(p, r, c.nn, rr_part, c.scal, parity, st);
    parity ^= 1;
}

constexpr int kCheck = 8;  // CG iterations per convergence poll

// CG on chi_Omega K chi_Omega from x with residual r (both in/out), for
// ||r|| / sqrt(bb) <= tol.  p, q: scratch.
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
    res.relres = sqrt(rr) / bn;
    if (res.relres <= tol) {
        res.converged = true;
        return res;
    }
    int parity = 0, it = 0;
    Poller pl(c, st);
    bool brk = false, hit = false;
    while (true) {
        const int nb = std::min(kCheck, maxit - it);
        for (int i = 0; i < nb; ++i) cg_iteration<T>(c, x, r, p, q, parity, matvecs, st);
        it += nb;
        pl.post(parity);
        bool done = false;
        if (it >= maxit) {
            pl.wait_last(rr, brk);
            done = true;
        } else if (pl.wait_prev(rr, brk)) {
            hit = std::isfinite(rr) && sqrt(rr) / bn <= tol;
            done = brk || hit || !std::isfinite(rr);
            if (done) {  // the batch in flight has run too
                double rr2;
                bool brk2;
                pl.wait_last(rr2, brk2);
                brk = brk || brk2;
                if (std::isfinite(rr2)) rr = hit ? std::min(rr, rr2) : rr2;
            }
        }
        if (done) break;
    }
    // the residual norm of CG is not monotone: convergence is the first poll at tol
    res.iters = it;
    res.relres = sqrt(rr) / bn;
    res.breakdown = brk || !std::isfinite(rr);
    res.converged = !res.breakdown && (hit || res.relres <= tol);
    return res;
}

template <typename TV>
void to_vec(const double* r, TV* out, long n, hipStream_t st)
{
    if constexpr (std::is_same_v<TV, float>) launch_to32(r, out, n, st);
    else HIPCHK(hipMemcpyAsync(out, r, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
}

template <typename TV>
void fold_into(double* x, TV* xc, long n, hipStream_t st)
{
    if constexpr (std::is_same_v<TV, float>) launch_add32to64_reset(x, xc, n, st);
    else {
        launch_add_reset64(x, xc, n, st);
    }
}

bool log_enabled()
{
    static int on = -1;
    if (on < 0) {
        const char* e = getenv("FCRKPM_LOG");
        on = (e && *e && *e != '0') ? 1 : 0;
    }
    return on == 1;
}

// CG with K products in FP32 and CG vectors of type TV; the solution x and
// the true residual are FP64.  The correction accumulates in xc (TV) and is
// folded into x, with the residual replaced by b - K x (FP64 products),
// whenever the recursive residual has fallen 10x since the last replacement.
// On entry v64[V_R] holds the true residual of x and inf.rel_res its norm.
template <typename TV>
fcrkpm_status reliable_cg(Ctx& c, TV* xc, TV* r, TV* p, TV* q, double bn, double tol, int maxit,
                          fcrkpm_info& inf, int& total, bool& need_f64,
                          const std::function<double()>& true_residual, hipStream_t st)
{
    const long nn = c.nn;
    double* x = c.v64 + 1 * nn;  // V_X
    double* r64 = c.v64 + 2 * nn;  // V_R
    const double drop2 = 1e-2;  // replace the residual when it fell 10x
    fcrkpm_status status = FCRKPM_OK;
    double rel = inf.rel_res;
    if (rel <= tol) return status;
    HIPCHK(hipMemsetAsync(xc, 0, sizeof(TV) * nn, st));
    HIPCHK(hipMemsetAsync(c.scal + S_BREAK, 0, sizeof(double), st));
    if ((void*)r != (void*)r64) to_vec<TV>(r64, r, nn, st);
    HIPCHK(hipMemcpyAsync(p, r, sizeof(TV) * nn, hipMemcpyDeviceToDevice, st));
    launch_dot_partial<TV>(r, r, nn, c.partial, st);
    launch_reduce_to(c.partial, c.scal + S_RR0, st);
    double rr_upd = read_scalar(c, S_RR0, st);
    int parity = 0, it = 0, stall = 0, it_upd = 0, longest = 0;
    double best = rel;
    Poller pl(c, st);
    while (true) {
        const int nb = std::min(kCheck, maxit - it);
        for (int i = 0; i < nb; ++i) cg_iteration<TV, float>(c, xc, r, p, q, parity, inf.matvecs_f32, st);
        it += nb;
        pl.post(parity);
        double rr = 0.0;
        bool brk = false;
        const bool have = pl.wait_prev(rr, brk);
        if (have && !std::isfinite(rr)) brk = true;
        const bool last = it >= maxit;
        // an interval far longer than every earlier one means the recursion
        // wanders at the accuracy floor of the FP32 products: replace anyway
        const bool overdue = it - it_upd > 3 * longest + 256;
        if (!last && !overdue &&
            !(have && (brk || rr <= drop2 * rr_upd || sqrt(rr) / bn <= tol)))
            continue;
        longest = std::max(longest, it - it_upd);
        it_upd = it;
        bool brk2 = false;
        pl.wait_last(rr, brk2);
        brk = brk || brk2 || !std::isfinite(rr);
        fold_into<TV>(x, xc, nn, st);
        rel = true_residual();
        inf.rel_res = rel;
        ++inf.outer_iters;
        if (log_enabled())
            fprintf(stderr, "[fcrkpm] replace %d at it %d: recursive %.3e true %.3e\n",
                    inf.outer_iters, it, sqrt(rr) / bn, rel);
        if (rel <= tol) break;
        if (last) {
            status = FCRKPM_ERR_NOCONV;
            break;
        }
        if (brk) {
            need_f64 = true;
            inf.fallback_used = 1;
            break;
        }
        if (rel > 0.5 * best) {
            if (++stall >= 3) {
                // the true residual stopped improving: within 4 tol this is the
                // attainable accuracy (rel_res reports it); otherwise finish
                // with FP64 CG
                if (best <= 4.0 * tol) break;
                need_f64 = true;
                inf.fallback_used = 1;
                break;
            }
        } else {
            stall = 0;
        }
        best = std::min(best, rel);
        if ((void*)r != (void*)r64) to_vec<TV>(r64, r, nn, st);
        launch_dot_partial<TV>(r, r, nn, c.partial, st);
        launch_reduce_to(c.partial, c.scal + parity, st);
        rr_upd = read_scalar(c, parity, st);
    }
    total += it;
    return status;
}

// Solve chi_Omega K chi_Omega x = b with b in v64[V_B] and the initial x in
// v64[V_X] (zero off the free nodes).  Returns status; fills info.
//
// FCRKPM_MODE_F32_REFINED: CG whose products and recurrences run in FP32 while
// the solution and the true residual are kept in FP64: the FP32 correction is
// folded into x (FP64) and the residual replaced by b - K x computed with FP64
// products whenever the recursive residual has fallen 10x since the last
// replacement ("reliable updates"), keeping the Krylov direction.  This is
// iterative refinement whose inner solver keeps its search space across outer
// steps.  Stagnation of the true residual falls back to FP64 CG.
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
        if (info) *info = inf;
        return FCRKPM_OK;
    }
    const double bn = sqrt(bb);
    int total = 0;
    bool need_f64 = (mode == FCRKPM_MODE_F64);
    std::function<double()> true_residual = [&]() {
        apply_one<double>(c, FCRKPM_OP_K, x, q, st);
        ++inf.matvecs_f64;
        launch_sub_masked(b, q, c.freem, r, nn, st);
        return sqrt(dot_to<double>(c, r, r, S_NORM, st)) / bn;
    };
    if (mode != FCRKPM_MODE_F64) inf.rel_res = true_residual();
    if (mode == FCRKPM_MODE_F32_REFINED) {
        status = reliable_cg<float>(c, c.v32 + 0 * nn, c.v32 + 1 * nn, c.v32 + 2 * nn,
                                    c.v32 + 3 * nn, bn, tol, maxit, inf, total, need_f64,
                                    true_residual, st);
    } else if (mode == FCRKPM_MODE_F32_PRODUCTS) {
        status = reliable_cg<double>(c, c.v64 + V_T * nn, r, p, q, bn, tol, maxit, inf, total,
                                     need_f64, true_residual, st);
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
    inf.true_rel_res = true_residual();
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
        c.basis_plan = build_plan(c, c.ex, c.s);
        SepPlan mom_plan = build_plan(c, c.ex2, c.nmono2);
        {
            // programs live in device memory: [basis p1 0..2, basis p2 0..2, moment p1 0..2]
            std::vector<SepProg> hp(9);
            for (int j = 0; j < 3; ++j) {
                hp[j] = c.basis_plan.p1[j];
                hp[3 + j] = c.basis_plan.p2[j];
                hp[6 + j] = mom_plan.p1[j];
            }
            c.dprog = dalloc<SepProg>(9);
            HIPCHK(hipMemcpy(c.dprog, hp.data(), sizeof(SepProg) * 9, hipMemcpyHostToDevice));
            for (int j = 0; j < 3; ++j) {
                c.basis_plan.d1[j] = c.dprog + j;
                c.basis_plan.d2[j] = c.dprog + 3 + j;
                mom_plan.d1[j] = c.dprog + 6 + j;
            }
        }
        {
            int dev = 0, maxsh = 0;
            HIPCHK(hipGetDevice(&dev));
            if (hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                maxsh > 0)
                c.lds_budget = maxsh;
            const size_t lds = std::max(sep_lds_need(c, c.basis_plan, 16), sep_lds_need(c, mom_plan, 16));
            if (lds > (size_t)std::min(c.lds_budget, 65536))
                fail(FCRKPM_ERR_UNSUPPORTED, "box too long for the LDS tiles of this basis");
        }

        // Alg 1: moment convolutions and per-node solves (FP64)
        c.b0_64 = dalloc<double>((size_t)c.s * nn);
        c.ba_64 = dalloc<double>((size_t)c.dim * c.s * nn);
        c.b0_32 = dalloc<float>((size_t)c.s * nn);
        c.ba_32 = dalloc<float>((size_t)c.dim * c.s * nn);
        {
            const int k = mom_plan.k;
            const int ng = (c.nmono2 + 1) / 2;
            cplx<double>* G = dalloc<cplx<double>>((size_t)(ng + 2 * mom_plan.maxpairs) * nn);
            cplx<double>* S1 = G + (size_t)ng * nn;
            cplx<double>* S2 = S1 + (size_t)mom_plan.maxpairs * nn;
            const void* src = nullptr;
            cplx<double>* dst = (k == 1) ? G : S1;
            for (int j = 0; j < k; ++j) {
                ProfScope ps(c, KD_SETUP_PASS, 0.0, st);
                launch_sep_pass<double, double>(c, c.axes[j], mom_plan.p1[j], mom_plan.d1[j],
                                                j == 0 ? SEP_LD_CHI : SEP_LD_PAIRS, src, c.chi,
                                                SEP_ST_PAIRS, dst, nullptr, nullptr, nullptr, st);
                src = dst;
                dst = (j + 2 == k) ? G : ((dst == S1) ? S2 : S1);
            }
            if (const char* dump = getenv("FCRKPM_DUMP")) {
                HIPCHK(hipStreamSynchronize(st));
                std::vector<cplx<double>> hg((size_t)ng * nn);
                HIPCHK(hipMemcpy(hg.data(), G, sizeof(cplx<double>) * hg.size(), hipMemcpyDeviceToHost));
                FILE* f = fopen((std::string(dump) + ".G.bin").c_str(), "wb");
                if (f) {
                    fwrite(hg.data(), sizeof(cplx<double>), hg.size(), f);
                    fclose(f);
                }
            }
            launch_moment_solve(c, G, c.dflag + 1, st);
            HIPCHK(hipMemcpyAsync(hflag, c.dflag, sizeof(hflag), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipGetLastError());
            dfree(G);
            if (hflag[1] != 0x7fffffff && !getenv("FCRKPM_DUMP"))
                fail(FCRKPM_ERR_SINGULAR, "moment matrix not positive definite at node " + std::to_string(hflag[1]));
        }

        // workspace: two slots of intermediate pair fields per precision
        c.work64 = dalloc<cplx<double>>((size_t)2 * c.basis_plan.maxpairs * nn);
        c.work32 = dalloc<cplx<float>>((size_t)2 * c.basis_plan.maxpairs * nn);
        c.v64 = dalloc<double>((size_t)6 * nn);
        c.v32 = dalloc<float>((size_t)5 * nn);
        c.partial = dalloc<double>(2 * kRedBlocks);
        c.scal = dalloc<double>(16);
        HIPCHK(hipMemsetAsync(c.scal, 0, 16 * sizeof(double), st));
        HIPCHK(hipHostMalloc((void**)&c.hscal, 16 * sizeof(double), hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&c.poll_ev[0], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c.poll_ev[1], hipEventDisableTiming));
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
        if (mode < FCRKPM_MODE_F64 || mode > FCRKPM_MODE_F32_PRODUCTS) fail(FCRKPM_ERR_ARG, "unknown mode");
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
        if (mode < FCRKPM_MODE_F64 || mode > FCRKPM_MODE_F32_PRODUCTS) fail(FCRKPM_ERR_ARG, "unknown mode");
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
    static std::string names[KD_NKINDS];
    if (kind < 0 || kind >= KD_NKINDS) return "";
    if (names[kind].empty()) names[kind] = kind_name(kind);
    return names[kind].c_str();
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
