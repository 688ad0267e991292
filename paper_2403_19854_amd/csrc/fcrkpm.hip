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
#include <memory>
#include <mutex>
#include <type_traits>
#include <string>
#include <utility>
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

// ------------------------------------------------- scratch of the allocation-free apply
// fcrkpm_apply_noalloc runs the passes of fcrkpm_apply with their workspace in
// this array instead of the context's.  Each GPU holds its own copy at its own
// address until the process ends; every call on one GPU shares it, so calls
// that overlap in time on one GPU race.  In host code `scratch` is a host-side
// stand-in: its device address comes from hipGetSymbolAddress, taken once per
// device by the setup call and kept per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch array
void* scratch_address()
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(FCRKPM_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// ------------------------------------------------------ kernel-duration sampler
// For each kernel kind, HIP events time the first kProfCap launches after
// sampling starts (recorded around the launch, or by the launch itself for
// the register passes); every launch is counted together with its
// algorithmic bytes (what the launch must read and write, from the array
// sizes).
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
        : p(c.prof_on && !c.capturing ? (Prof*)c.prof : nullptr), kind(kind_), st(st_)
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

void free_set(OpSet*& s)
{
    if (!s) return;
    dfree(s->ba_64);
    dfree(s->ba_32);
    dfree(s->cls);
    for (int l = 0; l < 2; ++l) {
        dfree(s->nbits[l]);
        dfree(s->noff[l]);
        dfree(s->nrec[l]);
    }
    sym_release_state(s->sym);
    delete s;
    s = nullptr;
}

void release(Ctx& c)
{
    sym_release(c);
    free_set(c.mass_set);
    free_set(c.shift_set);
    free_set(c.jac_set);
    dfree(c.chi);
    dfree(c.cls);
    dfree(c.freem);
    dfree(c.dirm);
    dfree(c.vol64);
    dfree(c.vol32);
    dfree(c.area64);
    dfree(c.area32);
    dfree(c.b0_64);
    dfree(c.ba_64);
    dfree(c.b0_32);
    dfree(c.ba_32);
    for (int a = 0; a < 3; ++a) {
        dfree(c.tw64[a]);
        dfree(c.tw32[a]);
        dfree(c.spec64[a]);
        dfree(c.spec32[a]);
        dfree(c.rtab32[a]);
        dfree(c.rtab64[a]);
    }
    dfree(c.work64);
    dfree(c.work32);
    dfree(c.v64);
    dfree(c.v32);
    dfree(c.partial);
    dfree(c.partial_wide);
    dfree(c.scal);
    dfree(c.act);
    dfree(c.nbits[0]);
    dfree(c.nbits[1]);
    dfree(c.noff[0]);
    dfree(c.noff[1]);
    dfree(c.nrec[0]);
    dfree(c.nrec[1]);
    dfree(c.dflag);
    if (c.aux) (void)hipStreamDestroy(c.aux);
    c.aux = nullptr;
    dfree(c.dprog);
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
    while (r % 7 == 0) {
        r /= 7;
        if (!push(7)) return false;
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
const T* area_of(const Ctx& c)
{
    if constexpr (sizeof(T) == 8) return c.area64;
    else return c.area32;
}

template <typename T>
int kind_of(int stage) { return stage + (sizeof(T) == 4 ? KD_STAGES : 0); }

// bytes of `nreal` real fields stored as complex pairs
template <typename T>
double pair_bytes(int nreal) { return (double)((nreal + 1) / 2) * sizeof(cplx<T>); }

// Pass workspace for nrhs right-hand sides (both precisions).
void ensure_work(Ctx& c, int nrhs)
{
    if (nrhs <= c.cap_work) return;
    if (c.capturing) fail(FCRKPM_ERR_ARG, "workspace cannot grow during graph capture");
    HIPCHK(hipDeviceSynchronize());
    dfree(c.work64);
    dfree(c.work32);
    c.cap_work = 0;
    const size_t per = (size_t)2 * c.basis_plan.maxpairs * c.nn;
    c.work64 = dalloc<cplx<double>>(per * nrhs);
    c.work32 = dalloc<cplx<float>>(per * nrhs);
    c.cap_work = nrhs;
}

// bytes between right-hand sides of a pair-field slot and of a real field
template <typename T>
long pair_rstride(const Ctx& c) { return (long)c.basis_plan.maxpairs * c.nn * (long)sizeof(cplx<T>); }
template <typename Tio>
long real_rstride(const Ctx& c) { return c.nn * (long)sizeof(Tio); }

// Part-1 passes on axes 0..k-2 (Alg 2/3 first half): the fields `in` (Tio,
// masked) become P_{k-2} pairs; returns the slot that holds them.
template <typename T, typename Tio>
cplx<T>* part1(Ctx& c, const SepPlan& sp, const Tio* in, const uint8_t* mask, cplx<T>* S1,
               cplx<T>* S2, int nrhs, hipStream_t st)
{
    const double nn = (double)c.nn * nrhs;
    const void* src = in;
    cplx<T>* dst = S1;
    for (int j = 0; j + 1 < sp.k; ++j) {
        const int ldm = (j == 0) ? SEP_LD_REAL : SEP_LD_PAIRS;
        const double inb = (j == 0) ? sizeof(Tio) + 1.0 : pair_bytes<T>(sp.size[j - 1]);
        RhsBatch rb{nrhs, j == 0 ? real_rstride<Tio>(c) : pair_rstride<T>(c), pair_rstride<T>(c), 0};
        ProfScope ps(c, kind_of<T>(KD_P1_X + c.axes[j]), nn * (inb + pair_bytes<T>(sp.size[j])), st);
        launch_sep_pass<T, Tio>(c, c.axes[j], sp.p1[j], sp.d1[j], ldm, src, mask, SEP_ST_PAIRS, dst, nullptr,
                                nullptr, nullptr, st, rb);
        src = dst;
        dst = (dst == S1) ? S2 : S1;
    }
    return (cplx<T>*)src;
}

// Part-2 passes on axes k-2..0 from P_{k-2} pairs in `cur` to the real fields
// `out` (masked).
template <typename T, typename Tio>
void part2(Ctx& c, const SepPlan& sp, cplx<T>* cur, cplx<T>* S1, cplx<T>* S2, Tio* out,
           const uint8_t* mask, int nrhs, hipStream_t st)
{
    const double nn = (double)c.nn * nrhs;
    for (int j = sp.k - 2; j >= 0; --j) {
        const double inb = pair_bytes<T>(sp.size[j]);
        if (j > 0) {
            cplx<T>* dst = (cur == S1) ? S2 : S1;
            RhsBatch rb{nrhs, pair_rstride<T>(c), pair_rstride<T>(c), 0};
            ProfScope ps(c, kind_of<T>(KD_P2_X + c.axes[j]), nn * (inb + pair_bytes<T>(sp.size[j - 1])), st);
            launch_sep_pass<T, Tio>(c, c.axes[j], sp.p2[j], sp.d2[j], SEP_LD_PAIRS, cur, nullptr, SEP_ST_PAIRS,
                                    dst, nullptr, nullptr, nullptr, st, rb);
            cur = dst;
        } else {
            RhsBatch rb{nrhs, pair_rstride<T>(c), real_rstride<Tio>(c), 0};
            ProfScope ps(c, kind_of<T>(KD_P2_X + c.axes[j]), nn * (inb + sizeof(Tio) + 1.0), st);
            launch_sep_pass<T, Tio>(c, c.axes[j], sp.p2[j], sp.d2[j], SEP_LD_PAIRS, cur, nullptr, SEP_ST_REAL,
                                    out, mask, nullptr, nullptr, st, rb);
        }
    }
}

// The register-resident FP32 K product applies to cubic boxes of the
// register-path lengths (the choice never depends on nrhs, so a batched
// product equals the single ones bit for bit).
bool use_reg_path(const Ctx& c, int /*nrhs*/)
{
    static int env = -1;
    if (env < 0) {
        const char* e = getenv("FCRKPM_REGPATH");
        env = (e && *e == '0') ? 0 : 1;
    }
    if (env != 1 || !c.use_regpath) return false;
    // 64^3 and 128^3 boxes: per-node records or the line-constant middle pass;
    // the other lengths (P x Q layouts, the 32-lane 256-point layout): the
    // line-constant pass only
    if (reg_path_ok(c)) return c.nrec[c.reg_layout] != nullptr;
    return reg_gpq_ok(c) && sym_active(c);
}

// Algorithmic bytes of one launch of each register-resident pass: the FP32
// fields it must read and write (masks 1 B per node), and in the middle pass
// the node-class bits and record offset (8 + 4 B per lane) and the records of
// the elements that are neither interior nor outside the domain (20 floats
// each).
double reg_pass_bytes(const Ctx& c, int k)
{
    const double nn = (double)c.nn;
    const double p0 = c.basis_plan.size[0], p1 = c.basis_plan.size[1];  // fields after x, after y
    switch (k) {
        case 0: return nn * (4 + 1 + p0 * 4 + (c.prof_pupd ? 4 + 4 : 0));
        case 1: return nn * (p0 * 4 + p1 * 4);
        case 2: {
            if (sym_active(c)) return sym_pass_bytes(c, 4);
            const double words = (double)reg_bits_words(c, c.reg_layout);
            return nn * (p1 * 4 + p1 * 4) + 12.0 * words +
                   (double)c.nload[c.reg_layout] * reg_record_floats(c) * 4;
        }
        case 3: return nn * (p1 * 4 + p0 * 4);
        default: return nn * (p0 * 4 + 1 + 4 + (c.prof_dot ? 4 : 0));
    }
}

void regprof_events(const void* cv, int k, hipEvent_t* e0, hipEvent_t* e1)
{
    Ctx& c = *(Ctx*)cv;
    static const int kinds[5] = {KD_P1_X, KD_P1_Y, KD_MID_K, KD_P2_Y, KD_P2_X};
    ProfKind& pk = ((Prof*)c.prof)->k[kind_of<float>(kinds[k])];
    ++pk.launches;
    pk.bytes += reg_pass_bytes(c, k) * c.prof_rhs;
    if (pk.nrec < kProfCap) {
        *e0 = pk.ev[2 * pk.nrec];
        *e1 = pk.ev[2 * pk.nrec + 1];
        ++pk.nrec;
    }
}

// the same for the FP64 register passes (8-byte fields)
double reg_pass_bytes64(const Ctx& c, int k)
{
    const double nn = (double)c.nn;
    const double p0 = c.basis_plan.size[0], p1 = c.basis_plan.size[1];
    switch (k) {
        case 0: return nn * (8 + 1 + p0 * 8);
        case 1: return nn * (p0 * 8 + p1 * 8);
        case 2: return sym_pass_bytes(c, 8);
        case 3: return nn * (p1 * 8 + p0 * 8);
        default: return nn * (p0 * 8 + 1 + 8 + (c.prof_dot ? 8 : 0));
    }
}

void regprof_events64(const void* cv, int k, hipEvent_t* e0, hipEvent_t* e1)
{
    Ctx& c = *(Ctx*)cv;
    static const int kinds[5] = {KD_P1_X, KD_P1_Y, KD_MID_K, KD_P2_Y, KD_P2_X};
    ProfKind& pk = ((Prof*)c.prof)->k[kind_of<double>(kinds[k])];
    ++pk.launches;
    pk.bytes += reg_pass_bytes64(c, k) * c.prof_rhs;
    if (pk.nrec < kProfCap) {
        *e0 = pk.ev[2 * pk.nrec];
        *e1 = pk.ev[2 * pk.nrec + 1];
        ++pk.nrec;
    }
}

bool use_reg_path64(const Ctx& c)
{
    static int env = -1;
    if (env < 0) {
        const char* e = getenv("FCRKPM_REGPATH64");
        env = (e && *e == '0') ? 0 : 1;
    }
    return env == 1 && c.use_regpath && reg_path64_ok(c);
}

void reg_k64(Ctx& c, const double* in, double* out, const uint8_t* mask, int nrhs, hipStream_t st,
             double* dot_part = nullptr, const double* dot_with = nullptr)
{
    ensure_work(c, nrhs);
    RegProf rp;
    if (c.prof_on && !c.capturing) {
        rp.c = &c;
        rp.events_fn = regprof_events64;
        c.prof_rhs = nrhs;
        c.prof_dot = dot_part != nullptr;
    }
    launch_reg_k64(c, in, out, mask, nrhs, dot_part, dot_with, st, rp);
}

void reg_k(Ctx& c, const float* in, float* out, const uint8_t* mask, int nrhs, hipStream_t st,
           double* dot_part = nullptr, const float* dot_with = nullptr, const RegPupd* pu = nullptr)
{
    ensure_work(c, nrhs);
    RegProf rp;
    if (c.prof_on && !c.capturing) {
        rp.c = &c;
        rp.events_fn = regprof_events;
        c.prof_rhs = nrhs;
        c.prof_dot = dot_part != nullptr;
    }
    c.prof_pupd = pu != nullptr;
    launch_reg_k(c, in, out, mask, nrhs, dot_part, dot_with, st, rp, pu);
}

void build_pointwise(Ctx& c, hipStream_t st);

// Exchanges the pointwise data of the K-type product in use with `s`.
void swap_set(Ctx& c, OpSet& s)
{
    std::swap(c.krows, s.krows);
    std::swap(c.ba_64, s.ba_64);
    std::swap(c.ba_32, s.ba_32);
    std::swap(c.cls, s.cls);
    std::swap(c.ncls2, s.ncls2);
    std::swap(c.cint64, s.cint64);
    std::swap(c.cint32, s.cint32);
    std::swap(c.nbits, s.nbits);
    std::swap(c.reg_mi, s.reg_mi);
    std::swap(c.noff, s.noff);
    std::swap(c.nrec, s.nrec);
    std::swap(c.nload, s.nload);
    std::swap(c.nconst, s.nconst);
    std::swap(c.sym, s.sym);
}

// The products of a scope use the set `s` (kernels take their arguments at
// launch, so the arrays only have to outlive the set).
struct SetScope {
    Ctx& c;
    OpSet* s;
    SetScope(Ctx& c_, OpSet* s_) : c(c_), s(s_) { if (s) swap_set(c, *s); }
    ~SetScope() { if (s) swap_set(c, *s); }
    SetScope(const SetScope&) = delete;
    SetScope& operator=(const SetScope&) = delete;
};

// Pointwise data of c_m M + c_k K (App. C): the rows sqrt(c_k) b^a of the
// stiffness (Eq 91) and sqrt(c_m) b^0 of the mass (Eq C.8), so that
// V sum_rows c_p c_q = V (c_k B^T B + c_m b^0 b^0T).  Synchronous.
OpSet* make_set(Ctx& c, double ck, double cm, hipStream_t st, const double* wnode = nullptr)
{
    if (c.capturing) fail(FCRKPM_ERR_ARG, "operator coefficients cannot be built during graph capture");
    if (!(ck >= 0.0) || !(cm >= 0.0) || !(ck > 0.0 || cm > 0.0) || !std::isfinite(ck) || !std::isfinite(cm))
        fail(FCRKPM_ERR_ARG, "operator weights must be finite, non-negative and not both zero");
    OpSet* s = new OpSet();
    s->krows = (ck > 0.0 ? c.dim : 0) + (cm > 0.0 ? 1 : 0);
    try {
        const size_t cnt = (size_t)s->krows * c.s * c.nn;
        s->ba_64 = dalloc<double>(cnt);
        s->ba_32 = dalloc<float>(cnt);
        launch_op_rows(c, ck, cm, s->ba_64, s->ba_32, st, wnode);
        HIPCHK(hipGetLastError());
        SetScope use(c, s);
        build_pointwise(c, st);
        // the line-constant middle pass, where this set's rows have the structure
        sym_build(c, st);
        HIPCHK(hipStreamSynchronize(st));
    } catch (...) {
        free_set(s);
        throw;
    }
    return s;
}

// the consistent mass M (Eq C.8), built on first use
OpSet* mass_set(Ctx& c, hipStream_t st)
{
    if (!c.mass_set) c.mass_set = make_set(c, 0.0, 1.0, st);
    return c.mass_set;
}

// c_m M + c_k K, rebuilt when the weights change
OpSet* shift_set(Ctx& c, double cm, double ck, hipStream_t st)
{
    if (!c.shift_set || c.shift_w[0] != cm || c.shift_w[1] != ck) {
        HIPCHK(hipStreamSynchronize(st));
        free_set(c.shift_set);
        c.shift_set = make_set(c, ck, cm, st);
        c.shift_w[0] = cm;
        c.shift_w[1] = ck;
    }
    return c.shift_set;
}

// internal operator: the passes of K_FULL with the gradient nonlinearity of
// c.pw_kappa between the two halves (Alg B.1 with N(g) = (1 + kappa |g|^2) g)
constexpr int OP_KN = 100;

// One operator on nrhs consecutive fields, arithmetic precision T, field type
// Tio (Alg 2, 3, 4, C.1, B.1); every pass covers all fields in one launch.
template <typename T, typename Tio = T>
void apply_one(Ctx& c, int op, const Tio* in, Tio* out, int nrhs, hipStream_t st)
{
    ensure_work(c, nrhs);
    const SepPlan& sp = c.basis_plan;
    const int k = sp.k, last = c.axes[k - 1];
    cplx<T>* S1 = work_of<T>(c);
    cplx<T>* S2 = S1 + (size_t)sp.maxpairs * c.nn * c.cap_work;
    const double nn = (double)c.nn * nrhs, rt = sizeof(T);
    const long prs = pair_rstride<T>(c), rrs = real_rstride<Tio>(c);
    const double inb1 = (k == 1) ? sizeof(Tio) + 1.0 : pair_bytes<T>(k >= 2 ? sp.size[k - 2] : 1);
    const double outb2 = (k == 1) ? sizeof(Tio) + 1.0 : pair_bytes<T>(k >= 2 ? sp.size[k - 2] : 1);
    switch (op) {
        case FCRKPM_OP_K:
        case FCRKPM_OP_K_FULL:
        case OP_KN: {
            const uint8_t* mk = (op == FCRKPM_OP_K) ? c.freem : c.chi;
            const int pwk = (op == OP_KN) ? SEP_PW_KN : SEP_PW_K;
            if constexpr (std::is_same_v<T, float> && std::is_same_v<Tio, float>) {
                if (op != OP_KN && use_reg_path(c, nrhs)) {
                    reg_k(c, in, out, mk, nrhs, st);
                    break;
                }
            }
            if constexpr (std::is_same_v<T, double> && std::is_same_v<Tio, double>) {
                if (op != OP_KN && use_reg_path64(c)) {
                    reg_k64(c, in, out, mk, nrhs, st);
                    break;
                }
                if (op == OP_KN && use_reg_path64(c) && reg_kn_ok(c, st)) {
                    for (int j = 0; j < nrhs; ++j)
                        launch_reg_kn(c, in + (size_t)j * c.nn, out + (size_t)j * c.nn, c.pw_kappa, RK_FORCE, st);
                    break;
                }
            }
            cplx<T>* cur = part1<T, Tio>(c, sp, in, mk, S1, S2, nrhs, st);
            cplx<T>* dst = (cur == S1) ? S2 : S1;
            {
                // coefficients are read only at class-2 nodes (1 B of class per node)
                const double coef = c.cls ? (double)c.ncls2 * (c.krows * c.s + 1) * rt + nn
                                          : nn * (c.krows * c.s + 1) * rt;
                ProfScope ps(c, kind_of<T>(KD_MID_K), nn * (inb1 + outb2) + coef, st);
                if (k == 1)
                    launch_sep_mid<T, Tio>(c, last, sp.p1[0], sp.d1[0], sp.p2[0], sp.d2[0], pwk, SEP_LD_REAL, in, mk,
                                           SEP_ST_REAL, out, mk, nullptr, b0_of<T>(c), ba_of<T>(c),
                                           vol_of<T>(c), nullptr, nullptr, st, RhsBatch{nrhs, rrs, rrs, 0});
                else
                    launch_sep_mid<T, Tio>(c, last, sp.p1[k - 1], sp.d1[k - 1], sp.p2[k - 1], sp.d2[k - 1], pwk, SEP_LD_PAIRS,
                                           cur, nullptr, SEP_ST_PAIRS, dst, nullptr, nullptr,
                                           b0_of<T>(c), ba_of<T>(c), vol_of<T>(c), nullptr, nullptr,
                                           st, RhsBatch{nrhs, prs, prs, 0});
            }
            if (k > 1) part2<T, Tio>(c, sp, dst, S1, S2, out, mk, nrhs, st);
            break;
        }
        case FCRKPM_OP_M: {
            // f^m = M d (Eq C.8, C.11; Alg C.1): the passes of K with the single
            // coefficient row b^0 and the domain mask on both sides
            SetScope use(c, mass_set(c, st));
            apply_one<T, Tio>(c, FCRKPM_OP_K_FULL, in, out, nrhs, st);
            break;
        }
        case FCRKPM_OP_FR:
        case FCRKPM_OP_NT:
        case FCRKPM_OP_UH:
        case FCRKPM_OP_VN:
        case FCRKPM_OP_FQ:
            if constexpr (!std::is_same_v<T, Tio>) {
                fail(FCRKPM_ERR_ARG, "mixed precisions are supported for K only");
            } else {
                if constexpr (std::is_same_v<T, double>) {
                    // u^h and f^r of one or more fields on the FP64 register path
                    if ((op == FCRKPM_OP_UH || op == FCRKPM_OP_FR) && use_reg_path64(c) && reg_kn_ok(c, st)) {
                        for (int j = 0; j < nrhs; ++j)
                            launch_reg_kn(c, in + (size_t)j * c.nn, out + (size_t)j * c.nn, 0.0,
                                          op == FCRKPM_OP_UH ? RK_UH : RK_LOAD, st);
                        break;
                    }
                }
                // f^q is the load pass of f^r with the boundary areas A in place
                // of V (Eq A.5, Alg A.1)
                if (op == FCRKPM_OP_FQ && !c.area64)
                    fail(FCRKPM_ERR_ARG, "no boundary areas: call fcrkpm_set_boundary first");
                const T* vol = (op == FCRKPM_OP_FR || op == FCRKPM_OP_VN) ? vol_of<T>(c)
                               : op == FCRKPM_OP_FQ                      ? area_of<T>(c)
                                                                         : nullptr;
                if (op == FCRKPM_OP_FR || op == FCRKPM_OP_NT || op == FCRKPM_OP_FQ) {
                    {
                        ProfScope ps(c, kind_of<T>(KD_MID_LOAD), nn * (sizeof(Tio) + (c.s + 1) * rt + outb2), st);
                        launch_sep_mid<T, Tio>(c, last, sp.p1[k - 1], sp.d1[k - 1], sp.p2[k - 1], sp.d2[k - 1], SEP_PW_LOAD,
                                               SEP_LD_PAIRS, nullptr, nullptr,
                                               k == 1 ? SEP_ST_REAL : SEP_ST_PAIRS,
                                               k == 1 ? (void*)out : (void*)S1, c.chi, in,
                                               b0_of<T>(c), ba_of<T>(c), vol, nullptr, nullptr, st,
                                               RhsBatch{nrhs, 0, k == 1 ? rrs : prs, rrs});
                    }
                    if (k > 1) part2<T, Tio>(c, sp, S1, S1, S2, out, c.chi, nrhs, st);
                } else {
                    cplx<T>* cur = part1<T, Tio>(c, sp, in, c.chi, S1, S2, nrhs, st);
                    ProfScope ps(c, kind_of<T>(KD_MID_UH), nn * (inb1 + (c.s + 1) * rt + sizeof(Tio)), st);
                    launch_sep_mid<T, Tio>(c, last, sp.p1[k - 1], sp.d1[k - 1], sp.p2[k - 1], sp.d2[k - 1], SEP_PW_UH,
                                           k == 1 ? SEP_LD_REAL : SEP_LD_PAIRS,
                                           k == 1 ? (const void*)in : (const void*)cur, c.chi,
                                           SEP_ST_REAL, out, nullptr, nullptr, b0_of<T>(c),
                                           ba_of<T>(c), vol, nullptr, nullptr, st,
                                           RhsBatch{nrhs, k == 1 ? rrs : prs, rrs, 0});
                }
            }
            break;
        default:
            fail(FCRKPM_ERR_ARG, "unknown operator");
    }
}

// ---------------------------------------------------------------- solvers
//
// Every solver works on nrhs right-hand sides at once: vector v of rhs j
// lives at v + j*nn inside blocks of cap_rhs fields, its device scalars at
// scal + j*kScal, and each launch covers all of them (blockIdx.y).  A rhs
// that has finished is frozen on the device (act[j] = 0) while the others
// keep iterating.

enum { V_B = 0, V_X = 1, V_R = 2, V_P = 3, V_Q = 4, V_T = 5 };
enum { S_RR0 = 0, S_RR1 = 1, S_BREAK = 3, S_NORM = 4, S_BB = 5 };

// Solver buffers for nrhs right-hand sides.  Never called during capture.
void ensure_rhs(Ctx& c, int nrhs)
{
    if (nrhs <= c.cap_rhs) return;
    if (c.capturing) fail(FCRKPM_ERR_ARG, "solver buffers cannot grow during graph capture");
    HIPCHK(hipDeviceSynchronize());
    dfree(c.v64);
    dfree(c.v32);
    dfree(c.partial);
    dfree(c.scal);
    dfree(c.act);
    if (c.hscal) (void)hipHostFree(c.hscal);
    c.hscal = nullptr;
    c.cap_rhs = 0;
    const size_t nn = (size_t)c.nn;
    c.v64 = dalloc<double>(6 * nn * nrhs);
    c.v32 = dalloc<float>(5 * nn * nrhs);
    c.partial = dalloc<double>((size_t)2 * kRedBlocks * nrhs);
    dfree(c.partial_wide);
    if (reg_dot_slots(c) > kRedBlocks) c.partial_wide = dalloc<double>((size_t)reg_dot_slots(c) * nrhs);
    c.scal = dalloc<double>((size_t)kScal * nrhs);
    c.act = dalloc<int>(nrhs);
    HIPCHK(hipMemset(c.scal, 0, sizeof(double) * kScal * nrhs));
    HIPCHK(hipMemset(c.act, 0, sizeof(int) * nrhs));
    HIPCHK(hipHostMalloc((void**)&c.hscal, sizeof(double) * 3 * kScal * nrhs, hipHostMallocDefault));
    c.cap_rhs = nrhs;
}

double* vec64(Ctx& c, int which) { return c.v64 + (size_t)which * c.nn * c.cap_rhs; }
float* vec32(Ctx& c, int which) { return c.v32 + (size_t)which * c.nn * c.cap_rhs; }

// scalars of all right-hand sides, read back synchronously
const double* read_scalars(Ctx& c, int nrhs, hipStream_t st)
{
    double* h = c.hscal + (size_t)2 * kScal * c.cap_rhs;
    HIPCHK(hipMemcpyAsync(h, c.scal, sizeof(double) * kScal * nrhs, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return h;
}

// scal[j*kScal + idx] = a_j . b_j for every right-hand side
template <typename T>
void dots(Ctx& c, const T* a, const T* b, int nrhs, int idx, hipStream_t st)
{
    launch_dot_partial<T>(a, b, c.nn, nrhs, c.partial, nullptr, st);
    launch_reduce_to(c.partial, c.nn, nrhs, c.scal + idx, st);
}

// the register-resident product can fold the CG direction update into its
// first pass (FP32 vectors and products only), and the p.q partials into its
// last pass where its workgroups fit the partial slots
template <typename T, typename TP>
bool fused_cg(Ctx& c, int nrhs)
{
    if constexpr (std::is_same_v<T, float> && std::is_same_v<TP, float>)
        return use_reg_path(c, nrhs);
    else
        return false;
}

// one CG iteration for all active right-hand sides: vectors of type T, K
// products in precision TP.  With `fused`, the product's first pass applies
// the direction update left pending by the previous iteration (pend) and this
// iteration leaves its own update pending unless `last`.
template <typename T, typename TP = T>
void cg_iteration(Ctx& c, T* x, T* r, T* p, T* q, int nrhs, int parity, hipStream_t st,
                  bool fused = false, bool pend = false, bool last = true)
{
    double* pq_part = c.partial;
    double* rr_part = c.partial + (size_t)kRedBlocks * c.cap_rhs;
    int npq = red_blocks(c.nn);
    if constexpr (std::is_same_v<T, float> && std::is_same_v<TP, float>) {
        if (fused) {
            // the last pass of the product also leaves the p.q partials (in
            // the wide slots, summed to one, when its workgroups outnumber
            // kRedBlocks)
            RegPupd pu{r, rr_part, red_blocks(c.nn), c.scal, parity ^ 1, c.act};
            const int nb = reg_path_blocks(c);
            const bool wide = nb > kRedBlocks;
            reg_k(c, p, q, c.freem, nrhs, st, wide ? c.partial_wide : pq_part, p, pend ? &pu : nullptr);
            npq = wide ? 1 : nb;
            if (wide) launch_reduce_wide(c.partial_wide, nb, reg_dot_slots(c), nrhs, pq_part, st);
        } else {
            apply_one<TP, T>(c, FCRKPM_OP_K, p, q, nrhs, st);
            launch_dot_partial<T>(p, q, c.nn, nrhs, pq_part, c.act, st);
        }
    } else if constexpr (std::is_same_v<T, double> && std::is_same_v<TP, double>) {
        if (use_reg_path64(c)) {
            // the last pass of the product leaves the p.q partials (wide
            // slots as in FP32)
            const int nb = (int)reg_path64_blocks(c);
            const bool wide = nb > kRedBlocks;
            reg_k64(c, p, q, c.freem, nrhs, st, wide ? c.partial_wide : pq_part, p);
            npq = wide ? 1 : nb;
            if (wide) launch_reduce_wide(c.partial_wide, nb, reg_dot_slots(c), nrhs, pq_part, st);
        } else {
            apply_one<TP, T>(c, FCRKPM_OP_K, p, q, nrhs, st);
            launch_dot_partial<T>(p, q, c.nn, nrhs, pq_part, c.act, st);
        }
    } else {
        apply_one<TP, T>(c, FCRKPM_OP_K, p, q, nrhs, st);
        launch_dot_partial<T>(p, q, c.nn, nrhs, pq_part, c.act, st);
    }
    launch_cg_xr<T>(x, r, p, q, c.nn, nrhs, pq_part, npq, c.scal, parity, rr_part, c.act, st);
    if (!fused || last) launch_cg_p<T>(p, r, c.nn, nrhs, rr_part, c.scal, parity, c.act, st);
}

constexpr int kCheck = 8;  // CG iterations per convergence poll (even: parity returns)

bool log_enabled()
{
    static int on = -1;
    if (on < 0) {
        const char* e = getenv("FCRKPM_LOG");
        on = (e && *e && *e != '0') ? 1 : 0;
    }
    return on == 1;
}

struct RhsState {
    double bn = 1.0;       // ||b_j||
    double rel = 0.0;      // relative residual reported (true one in refinement)
    double best = 0.0;     // best true residual seen by refinement
    double rr_upd = 0.0;   // recursive r.r right after the last replacement
    double rr_poll = 0.0;  // r.r of the last look-ahead poll
    double rr_last = 0.0;  // recursive r.r when the last block ended
    int iters = 0, outer = 0, stall = 0, it_upd = 0, longest = 0;
    int mv32 = 0, mv64 = 0;
    bool active = false;   // iterating in the current phase
    bool want = false;     // asked for service at the last poll
    bool hit = false;      // FP64 phase: recursive residual at tol at the last poll
    bool brk = false;
    bool conv = false;
    bool need64 = false;   // refinement handed it to FP64 CG
    bool fallback = false;
    bool zero = false;     // b = 0
};

enum Phase { PH_REFINED, PH_F64, PH_DONE };

// Strong-Dirichlet CG on chi_Omega K chi_Omega x = b for nrhs right-hand
// sides (Alg 5), b in vec64(V_B), the initial x in vec64(V_X).
//
// FCRKPM_MODE_F32_REFINED: CG whose products and recurrences run in FP32
// while the solution and the true residual are kept in FP64: the FP32
// correction is folded into x (FP64) and the residual replaced by b - K x
// computed with FP64 products whenever the recursive residual has fallen 10x
// since the last replacement ("reliable updates"), keeping the Krylov
// direction.  This is iterative refinement whose inner solver keeps its
// search space across outer steps.  A right-hand side whose true residual
// stagnates finishes with FP64 CG.
// FCRKPM_MODE_F32_PRODUCTS: the same with FP64 vectors and FP32 products.
// FCRKPM_MODE_F64: plain FP64 CG.
//
// The driver (run_solvers) enqueues blocks of kCheck iterations, posts the
// scalars after each block and calls wants()/service() from the host.
struct Solver {
    Ctx& c;
    int nrhs, mode, maxit;
    double tol;
    Phase ph = PH_DONE;
    int it = 0;           // iterations in the current phase
    int it_base = 0;      // iterations spent before the current phase
    int parity = 0;       // slot of r.r the next iteration reads
    int parity_of[2] = {0, 0};
    std::vector<RhsState> R;
    hipEvent_t join = nullptr;
    const double drop2 = 1e-2;  // replace the residual when it fell 10x

    Solver(Ctx& c_, int nrhs_, int mode_, double tol_, int maxit_)
        : c(c_), nrhs(nrhs_), mode(mode_), maxit(maxit_), tol(tol_), R(nrhs_)
    {
        HIPCHK(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    }
    ~Solver()
    {
        if (join) (void)hipEventDestroy(join);
    }

    int phase_maxit() const { return std::max(1, maxit - it_base); }
    bool any_active() const
    {
        for (const auto& s : R)
            if (s.active) return true;
        return false;
    }

    // b - K x into vec64(V_R) for all rhs; returns after reading the norms
    void true_residual(hipStream_t st)
    {
        double* b = vec64(c, V_B);
        double* x = vec64(c, V_X);
        double* r = vec64(c, V_R);
        double* q = vec64(c, V_Q);
        apply_one<double>(c, FCRKPM_OP_K, x, q, nrhs, st);
        launch_sub_masked(b, q, c.freem, r, c.nn, nrhs, st);
        dots<double>(c, r, r, nrhs, S_NORM, st);
        const double* h = read_scalars(c, nrhs, st);
        for (int j = 0; j < nrhs; ++j) {
            ++R[j].mv64;
            R[j].rel = R[j].zero ? 0.0 : sqrt(h[j * kScal + S_NORM]) / R[j].bn;
        }
    }

    void set_flags(hipStream_t st)
    {
        for (int j = 0; j < nrhs; ++j) launch_set_flag(c.act, j, R[j].active ? 1 : 0, st);
    }

    void begin(hipStream_t st)
    {
        const long nn = c.nn;
        dots<double>(c, vec64(c, V_B), vec64(c, V_B), nrhs, S_BB, st);
        const double* h = read_scalars(c, nrhs, st);
        for (int j = 0; j < nrhs; ++j) {
            const double bb = h[j * kScal + S_BB];
            R[j].zero = !(bb > 0.0);
            R[j].bn = R[j].zero ? 1.0 : sqrt(bb);
            if (R[j].zero) {
                HIPCHK(hipMemsetAsync(vec64(c, V_X) + j * nn, 0, sizeof(double) * nn, st));
                R[j].conv = true;
            }
        }
        true_residual(st);
        if (mode == FCRKPM_MODE_F64) {
            for (auto& s : R) s.need64 = !s.zero;
            start_f64(st);
            return;
        }
        // FP32 refinement keeps its best iterate in vec64(V_T)
        if (mode == FCRKPM_MODE_F32_REFINED)
            HIPCHK(hipMemcpyAsync(vec64(c, V_T), vec64(c, V_X), sizeof(double) * nn * nrhs,
                                  hipMemcpyDeviceToDevice, st));
        bool any = false;
        for (auto& s : R) {
            s.best = s.rel;
            s.active = !s.zero && s.rel > tol;
            if (!s.zero && !s.active) s.conv = true;
            any = any || s.active;
        }
        if (!any) {
            ph = PH_DONE;
            return;
        }
        ph = PH_REFINED;
        it = 0;
        parity = 0;
        launch_set_scalar(c.scal, S_BREAK, 0.0, nrhs, st);
        if (mode == FCRKPM_MODE_F32_REFINED) {
            HIPCHK(hipMemsetAsync(vec32(c, 0), 0, sizeof(float) * nn * nrhs, st));
            launch_to32(vec64(c, V_R), vec32(c, 1), nn * nrhs, st);
            HIPCHK(hipMemcpyAsync(vec32(c, 2), vec32(c, 1), sizeof(float) * nn * nrhs,
                                  hipMemcpyDeviceToDevice, st));
            dots<float>(c, vec32(c, 1), vec32(c, 1), nrhs, S_RR0, st);
        } else {
            HIPCHK(hipMemsetAsync(vec64(c, V_T), 0, sizeof(double) * nn * nrhs, st));
            HIPCHK(hipMemcpyAsync(vec64(c, V_P), vec64(c, V_R), sizeof(double) * nn * nrhs,
                                  hipMemcpyDeviceToDevice, st));
            dots<double>(c, vec64(c, V_R), vec64(c, V_R), nrhs, S_RR0, st);
        }
        h = read_scalars(c, nrhs, st);
        for (int j = 0; j < nrhs; ++j) R[j].rr_upd = h[j * kScal + S_RR0];
        set_flags(st);
    }

    // FP64 CG from the current x with r = b - K x already in vec64(V_R), for
    // the rhs marked need64
    void start_f64(hipStream_t st)
    {
        const long nn = c.nn;
        it_base += it;
        it = 0;
        parity = 0;
        ph = PH_F64;
        HIPCHK(hipMemcpyAsync(vec64(c, V_P), vec64(c, V_R), sizeof(double) * nn * nrhs,
                              hipMemcpyDeviceToDevice, st));
        launch_set_scalar(c.scal, S_BREAK, 0.0, nrhs, st);
        dots<double>(c, vec64(c, V_R), vec64(c, V_R), nrhs, S_RR0, st);
        const double* h = read_scalars(c, nrhs, st);
        bool any = false;
        for (int j = 0; j < nrhs; ++j) {
            RhsState& s = R[j];
            s.active = false;
            if (!s.need64) continue;
            s.rel = sqrt(h[j * kScal + S_RR0]) / s.bn;
            if (s.rel <= tol) {
                s.conv = true;
                continue;
            }
            s.active = true;
            any = true;
        }
        if (!any) {
            ph = PH_DONE;
            return;
        }
        set_flags(st);
    }

    // kCheck (or fewer) iterations of the current phase: kernel launches only,
    // so the block can be captured into a graph and replayed
    void enqueue(int nb, hipStream_t st)
    {
        int par = parity;
        const bool fused = ph == PH_REFINED && mode == FCRKPM_MODE_F32_REFINED &&
                           fused_cg<float, float>(c, nrhs);
        for (int i = 0; i < nb; ++i, par ^= 1) {
            if (ph == PH_F64)
                cg_iteration<double>(c, vec64(c, V_X), vec64(c, V_R), vec64(c, V_P), vec64(c, V_Q),
                                     nrhs, par, st);
            else if (mode == FCRKPM_MODE_F32_REFINED)
                // within a block the direction update of iteration i runs in the
                // first pass of iteration i+1; the block ends with it applied
                cg_iteration<float, float>(c, vec32(c, 0), vec32(c, 1), vec32(c, 2), vec32(c, 3),
                                           nrhs, par, st, fused, i > 0, i == nb - 1);
            else
                cg_iteration<double, float>(c, vec64(c, V_T), vec64(c, V_R), vec64(c, V_P),
                                            vec64(c, V_Q), nrhs, par, st);
        }
    }

    // bookkeeping of an enqueued block
    void advance(int nb)
    {
        it += nb;
        parity ^= (nb & 1);
        for (auto& s : R)
            if (s.active) {
                s.iters += nb;
                if (ph == PH_F64) s.mv64 += nb;
                else s.mv32 += nb;
            }
    }

    void post(int slot, hipStream_t st)
    {
        HIPCHK(hipMemcpyAsync(c.hscal + (size_t)slot * kScal * c.cap_rhs, c.scal,
                              sizeof(double) * kScal * nrhs, hipMemcpyDeviceToHost, st));
        parity_of[slot] = parity;
    }

    // from the scalars of a completed post: does any rhs need the host?
    bool wants(int slot)
    {
        const double* h = c.hscal + (size_t)slot * kScal * c.cap_rhs;
        const int pp = parity_of[slot];
        bool any = it >= phase_maxit();
        for (int j = 0; j < nrhs; ++j) {
            RhsState& s = R[j];
            s.want = false;
            if (!s.active) continue;
            const double rr = h[j * kScal + pp];
            const bool brk = h[j * kScal + S_BREAK] != 0.0 || !std::isfinite(rr);
            s.rr_poll = rr;
            if (ph == PH_REFINED) {
                const bool overdue = it - s.it_upd > 3 * s.longest + 256;
                s.want = brk || rr <= drop2 * s.rr_upd || sqrt(rr) / s.bn <= tol || overdue;
                s.brk = brk;
            } else {
                s.hit = std::isfinite(rr) && sqrt(rr) / s.bn <= tol;
                s.brk = brk;
                s.want = brk || s.hit;
            }
            any = any || s.want;
        }
        return any;
    }

    // host work after every posted block has completed; `slot` holds the
    // scalars of the last one
    void service(int slot, hipStream_t st)
    {
        const double* h = c.hscal + (size_t)slot * kScal * c.cap_rhs;
        const int pp = parity_of[slot];
        const bool last = it >= phase_maxit();
        bool any_want = false;
        for (const auto& s : R) any_want = any_want || (s.active && s.want);
        if (!any_want && !last) return;
        const long nn = c.nn;
        if (ph == PH_REFINED) {
            for (int j = 0; j < nrhs; ++j) {
                RhsState& s = R[j];
                if (!s.active) continue;
                const double rr2 = h[j * kScal + pp];
                s.rr_last = rr2;
                s.brk = s.brk || h[j * kScal + S_BREAK] != 0.0 || !std::isfinite(rr2);
            }
            if (mode == FCRKPM_MODE_F32_REFINED)
                launch_add32to64_reset(vec64(c, V_X), vec32(c, 0), nn * nrhs, st);
            else
                launch_add_reset64(vec64(c, V_X), vec64(c, V_T), nn * nrhs, st);
            std::vector<double> before(nrhs);
            for (int j = 0; j < nrhs; ++j) before[j] = R[j].rel;
            true_residual(st);
            bool any = false, need64 = false;
            std::vector<int> restart, restore;
            const bool keep = mode == FCRKPM_MODE_F32_REFINED;
            for (int j = 0; j < nrhs; ++j) {
                RhsState& s = R[j];
                if (!s.active) {
                    s.rel = before[j];  // frozen: keep what it finished with
                    continue;
                }
                const bool improved = s.rel < s.best;
                if (keep && improved)
                    HIPCHK(hipMemcpyAsync(vec64(c, V_T) + j * nn, vec64(c, V_X) + j * nn,
                                          sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
                // the FP32 recursion has left the true residual far behind (its
                // search direction no longer fits): restart it from the new
                // residual instead of keeping the direction
                const double true_rr = (s.rel * s.bn) * (s.rel * s.bn);
                const bool drifted = true_rr > 100.0 * s.rr_last;
                ++s.outer;
                if (s.want || last) s.longest = std::max(s.longest, it - s.it_upd);
                s.it_upd = it;
                if (log_enabled())
                    fprintf(stderr, "[fcrkpm] rhs %d replace %d at it %d: true %.3e\n", j, s.outer,
                            it, s.rel);
                if (s.rel <= tol) {
                    s.conv = true;
                    s.active = false;
                } else if (last) {
                    s.active = false;
                } else if (s.brk || s.rel > 10.0 * s.best) {
                    // breakdown, or the FP32 iteration diverged: finish in FP64
                    s.need64 = s.fallback = true;
                    s.active = false;
                } else if (s.want && s.rel > 0.5 * s.best) {
                    if (++s.stall >= 3) {
                        // the true residual stopped improving: within 4 tol this is
                        // the attainable accuracy; otherwise finish with FP64 CG
                        if (s.best <= 4.0 * tol) s.conv = true;
                        else s.need64 = s.fallback = true;
                        s.active = false;
                    }
                } else if (s.want) {
                    s.stall = 0;
                }
                // stopping (converged by stall, handed to FP64 or out of
                // iterations) on an iterate worse than the best: go back to it
                if (keep && !s.active && !improved && s.rel > s.best) restore.push_back(j);
                s.best = std::min(s.best, s.rel);
                s.want = false;
                if (s.active && drifted) restart.push_back(j);
                any = any || s.active;
                need64 = need64 || s.need64;
            }
            if (!restore.empty()) {
                for (int j : restore)
                    HIPCHK(hipMemcpyAsync(vec64(c, V_X) + j * nn, vec64(c, V_T) + j * nn,
                                          sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
                std::vector<double> kept(nrhs);
                for (int j = 0; j < nrhs; ++j) kept[j] = R[j].rel;
                true_residual(st);  // V_R = b - K x for the FP64 phase
                std::vector<bool> back(nrhs, false);
                for (int j : restore) back[j] = true;
                for (int j = 0; j < nrhs; ++j)
                    if (!back[j]) R[j].rel = kept[j];
                if (log_enabled())
                    for (int j : restore)
                        fprintf(stderr, "[fcrkpm] rhs %d back to its best iterate: true %.3e\n", j,
                                R[j].rel);
            }
            if (any) {
                if (mode == FCRKPM_MODE_F32_REFINED) {
                    launch_to32(vec64(c, V_R), vec32(c, 1), nn * nrhs, st);
                    for (int j : restart)
                        HIPCHK(hipMemcpyAsync(vec32(c, 2) + j * nn, vec32(c, 1) + j * nn,
                                              sizeof(float) * nn, hipMemcpyDeviceToDevice, st));
                    dots<float>(c, vec32(c, 1), vec32(c, 1), nrhs, parity, st);
                } else {
                    for (int j : restart)
                        HIPCHK(hipMemcpyAsync(vec64(c, V_P) + j * nn, vec64(c, V_R) + j * nn,
                                              sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
                    dots<double>(c, vec64(c, V_R), vec64(c, V_R), nrhs, parity, st);
                }
                if (log_enabled())
                    for (int j : restart) fprintf(stderr, "[fcrkpm] rhs %d restarts at it %d\n", j, it);
                const double* hr = read_scalars(c, nrhs, st);
                for (int j = 0; j < nrhs; ++j)
                    if (R[j].active) R[j].rr_upd = hr[j * kScal + parity];
                set_flags(st);
            } else if (need64 && !last) {
                start_f64(st);
            } else {
                ph = PH_DONE;
            }
        } else {
            bool any = false;
            for (int j = 0; j < nrhs; ++j) {
                RhsState& s = R[j];
                if (!s.active) continue;
                if (s.want || last) {
                    const double rr2 = h[j * kScal + pp];
                    const bool brk2 = h[j * kScal + S_BREAK] != 0.0;
                    s.brk = s.brk || brk2 || (!s.hit && !std::isfinite(rr2));
                    double rr = s.want ? s.rr_poll : rr2;
                    if (std::isfinite(rr2)) rr = s.hit ? std::min(s.rr_poll, rr2) : rr2;
                    // the residual norm of CG is not monotone: convergence is the
                    // first poll at tol
                    s.rel = sqrt(rr) / s.bn;
                    s.conv = !s.brk && (s.hit || s.rel <= tol);
                    s.active = false;
                }
                s.want = false;
                any = any || s.active;
            }
            if (any) set_flags(st);
            else ph = PH_DONE;
        }
    }

    // final true residuals and info; status of the worst rhs
    fcrkpm_status finish(fcrkpm_info* info, hipStream_t st)
    {
        std::vector<double> rel(nrhs);
        for (int j = 0; j < nrhs; ++j) rel[j] = R[j].rel;
        true_residual(st);
        fcrkpm_status status = FCRKPM_OK;
        for (int j = 0; j < nrhs; ++j) {
            RhsState& s = R[j];
            // refinement converges on the true residual: a final one far above
            // tol (an FP64 finish whose recursion lost it) is not convergence
            if (mode != FCRKPM_MODE_F64 && s.conv && !(s.rel <= 100.0 * tol)) s.conv = false;
            if (!s.conv) status = FCRKPM_ERR_NOCONV;
            if (info) {
                fcrkpm_info& f = info[j];
                memset(&f, 0, sizeof(f));
                f.iters = s.iters;
                f.outer_iters = s.outer;
                f.rel_res = rel[j];
                f.true_rel_res = s.rel;
                f.fallback_used = s.fallback ? 1 : 0;
                f.matvecs_f64 = s.mv64;
                f.matvecs_f32 = s.mv32;
            }
        }
        return status;
    }
};

bool graphs_enabled(const Ctx& c)
{
    if (c.prof_on || !c.use_graphs) return false;
    static int env = -1;
    if (env < 0) {
        const char* e = getenv("FCRKPM_GRAPHS");
        env = (e && *e == '0') ? 0 : 1;
    }
    return env == 1;
}

// Enqueue one block for every solver in `act`: a single one on `st`, several
// on their own streams forked from and joined back into `st`.
void enqueue_all(const std::vector<Solver*>& act, int nb, hipEvent_t fork, hipStream_t st)
{
    if (act.size() == 1) {
        act[0]->enqueue(nb, st);
        return;
    }
    HIPCHK(hipEventRecord(fork, st));
    for (Solver* s : act) {
        if (!s->c.aux) HIPCHK(hipStreamCreateWithFlags(&s->c.aux, hipStreamNonBlocking));
        HIPCHK(hipStreamWaitEvent(s->c.aux, fork, 0));
        s->enqueue(nb, s->c.aux);
        HIPCHK(hipEventRecord(s->join, s->c.aux));
    }
    for (Solver* s : act) HIPCHK(hipStreamWaitEvent(st, s->join, 0));
}

// Drive solvers to completion.  Blocks of kCheck iterations of every
// unfinished solver are enqueued together -- replayed from one captured HIP
// graph while the set of solvers and their phases stay the same -- and after
// each block the device scalars are copied to a pinned slot and an event is
// recorded.  The host only waits for the block before the one in flight
// (look-ahead), so the queue does not drain while it decides.
void run_solvers_on(const std::vector<Solver*>& all, bool graphs, hipStream_t st);

void run_solvers(const std::vector<Solver*>& all, bool graphs, hipStream_t st)
{
    if (!graphs || st != nullptr) {
        run_solvers_on(all, graphs, st);
        return;
    }
    // the legacy null stream cannot be captured: run on a private stream
    // ordered after everything enqueued so far
    HIPCHK(hipStreamSynchronize(st));
    hipStream_t own = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    try {
        run_solvers_on(all, graphs, own);
    } catch (...) {
        (void)hipStreamSynchronize(own);
        (void)hipStreamDestroy(own);
        throw;
    }
    HIPCHK(hipStreamSynchronize(own));
    HIPCHK(hipStreamDestroy(own));
}

void run_solvers_on(const std::vector<Solver*>& all, bool graphs, hipStream_t st)
{
    for (Solver* s : all) s->begin(st);
    hipEvent_t ev[2] = {nullptr, nullptr}, fork = nullptr;
    hipGraphExec_t ge = nullptr;
    std::vector<std::pair<Solver*, int>> gkey;
    auto cleanup = [&]() {
        for (Solver* s : all) s->c.capturing = false;
        if (ge) (void)hipGraphExecDestroy(ge);
        ge = nullptr;
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        ev[0] = ev[1] = fork = nullptr;
    };
    try {
        HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        int slot = 0, nposted = 0;
        while (true) {
            std::vector<Solver*> act;
            for (Solver* s : all)
                if (s->ph != PH_DONE) act.push_back(s);
            if (act.empty()) break;
            int nb = kCheck;
            for (Solver* s : act) nb = std::min(nb, s->phase_maxit() - s->it);
            nb = std::max(nb, 1);
            if (graphs && nb == kCheck) {
                std::vector<std::pair<Solver*, int>> key;
                for (Solver* s : act) key.emplace_back(s, (int)s->ph * 2 + s->parity);
                if (key != gkey || !ge) {
                    if (ge) {
                        HIPCHK(hipStreamSynchronize(st));
                        HIPCHK(hipGraphExecDestroy(ge));
                    }
                    ge = nullptr;
                    hipGraph_t g = nullptr;
                    for (Solver* s : act) s->c.capturing = true;
                    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                    try {
                        enqueue_all(act, nb, fork, st);
                    } catch (...) {
                        (void)hipStreamEndCapture(st, &g);
                        if (g) (void)hipGraphDestroy(g);
                        throw;
                    }
                    HIPCHK(hipStreamEndCapture(st, &g));
                    for (Solver* s : act) s->c.capturing = false;
                    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    HIPCHK(e);
                    gkey = key;
                }
                HIPCHK(hipGraphLaunch(ge, st));
            } else {
                enqueue_all(act, nb, fork, st);
            }
            for (Solver* s : act) {
                s->advance(nb);
                s->post(slot, st);
            }
            HIPCHK(hipEventRecord(ev[slot], st));
            slot ^= 1;
            ++nposted;
            bool need = false;
            if (nposted >= 2) {
                HIPCHK(hipEventSynchronize(ev[slot]));  // the block before the one in flight
                for (Solver* s : act) need = s->wants(slot) || need;
            } else {
                for (Solver* s : act) need = need || s->it >= s->phase_maxit();
            }
            if (need) {
                HIPCHK(hipEventSynchronize(ev[slot ^ 1]));
                for (Solver* s : act) s->service(slot ^ 1, st);
                nposted = 0;
            }
        }
    } catch (...) {
        (void)hipStreamSynchronize(st);
        cleanup();
        throw;
    }
    cleanup();
}

}  // namespace

[[noreturn]] void fcrkpm::raise_unsupported(const char* msg) { fail(FCRKPM_ERR_UNSUPPORTED, msg); }

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

namespace {
// Autotuner of the register-resident K passes: time a few FP32 K products
// with each variant -- line layout (8 or 16 lanes) times tiles per workgroup
// (1 or 2) -- on this device and keep the fastest.  FCRKPM_REGLAYOUT=v in the
// environment forces variant v = layout + 2 (tiles - 1).
// Node classes and the pointwise data of the K-type product whose coefficient
// rows c.ba_64 (c.krows of them) are in place: classes 0 outside the domain,
// 1 interior, 2 other; the interior constants; and the register-path bits and
// records.  The quadratic register records hold the rows b^a themselves, so
// they serve K alone.
void build_pointwise(Ctx& c, hipStream_t st)
{
    const long nn = c.nn;
    // node classes (0 outside the domain, 1 interior, 2 other) for the
    // pointwise stage of the K products: interior nodes share the first
    // interior node's b^a and V, nodes outside have V = 0
    if (c.krows * c.s <= kMaxNodeConst) {
        int big = 0x7fffffff, ref = 0;
        HIPCHK(hipMemcpyAsync(c.dflag + 3, &big, sizeof(int), hipMemcpyHostToDevice, st));
        launch_first_interior(c, c.dflag + 3, st);
        HIPCHK(hipMemcpyAsync(&ref, c.dflag + 3, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const int nb = c.krows * c.s;
        NodeConst nc = {};
        nc.bmax = -1.0;  // no interior node: every domain node is class 2
        if (ref != 0x7fffffff) {
            for (int q = 0; q < nb; ++q)
                HIPCHK(hipMemcpy(&nc.b[q], c.ba_64 + (size_t)q * nn + ref, sizeof(double),
                                 hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(&nc.v, c.vol64 + ref, sizeof(double), hipMemcpyDeviceToHost));
            nc.bmax = 0.0;
            for (int q = 0; q < nb; ++q) nc.bmax = std::max(nc.bmax, fabs(nc.b[q]));
        }
        c.cls = dalloc<uint8_t>(nn);
        launch_node_class(c, nc, c.cls, st);
        {
            std::vector<uint8_t> hc(nn);
            HIPCHK(hipMemcpyAsync(hc.data(), c.cls, nn, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            c.ncls2 = (long)std::count(hc.begin(), hc.end(), (uint8_t)2);
        }
        c.nconst = nc;
        for (int q = 0; q < nb; ++q) {
            c.cint64[q] = nc.b[q];
            c.cint32[q] = (float)nc.b[q];
        }
        c.cint64[nb] = nc.v;
        c.cint32[nb] = (float)nc.v;
    }
    // node classes of the register-resident K passes: interior nodes share
    // one M = V B^T B (a kernel argument), nodes outside the domain give
    // zero, and every other element gets its own record, packed lane by lane
    if (reg_path_ok(c) && c.cls && (c.degree == 1 || c.krows == c.dim)) {
        const uint8_t* cls = c.cls;
        const NodeConst& nc = c.nconst;
        if (nc.bmax >= 0.0 && c.degree == 1) {
            int k = 0;
            for (int p = 0; p < c.s; ++p)
                for (int q = p; q < c.s; ++q) {
                    double acc = 0.0;
                    for (int al = 0; al < c.krows; ++al) acc += nc.b[al * c.s + p] * nc.b[al * c.s + q];
                    c.reg_mi[k++] = (float)(nc.v * acc);
                }
        }
        const int rf = reg_record_floats(c);
        unsigned long long* cnt = reinterpret_cast<unsigned long long*>(c.dflag + 4);
        for (int lay = 0; lay < reg_layouts(c); ++lay) {
            const long words = reg_bits_words(c, lay);
            c.nbits[lay] = dalloc<uint2>(words);
            c.noff[lay] = dalloc<uint32_t>(words);
            unsigned long long zero = 0, got = 0;
            HIPCHK(hipMemcpyAsync(cnt, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
            launch_reg_bits(c, lay, cls, c.nbits[lay], c.noff[lay], cnt, st);
            HIPCHK(hipMemcpyAsync(&got, cnt, sizeof(got), hipMemcpyDeviceToHost, st));
            std::vector<uint32_t> off(words);
            HIPCHK(hipMemcpyAsync(off.data(), c.noff[lay], sizeof(uint32_t) * words,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            c.nload[lay] = (long)got;
            // per-lane counts -> first record of each lane (exclusive prefix sum)
            uint64_t run = 0;
            for (long s = 0; s < words; ++s) {
                const uint32_t n1 = off[s];
                off[s] = (uint32_t)run;
                run += n1;
            }
            if (run != got || run > 0xffffffffull) fail(FCRKPM_ERR_HIP, "record count mismatch");
            HIPCHK(hipMemcpyAsync(c.noff[lay], off.data(), sizeof(uint32_t) * words,
                                  hipMemcpyHostToDevice, st));
            c.nrec[lay] = dalloc<float>((size_t)std::max<uint64_t>(run, 1) * rf);
            launch_reg_recs(c, lay, c.nbits[lay], c.noff[lay], c.nrec[lay], st);
            HIPCHK(hipStreamSynchronize(st));
        }
    }
}

void set_reg_variant(Ctx& c, int v)
{
    c.reg_layout = v & 1;
    c.reg_tpw = (v >> 1) + 1;
}

void tune_reg_layout(Ctx& c, hipStream_t st)
{
    if (!use_reg_path(c, 1)) return;
    float* x = vec32(c, 2);
    float* y = vec32(c, 3);
    HIPCHK(hipMemsetAsync(x, 0, sizeof(float) * c.nn, st));
    // the trial launches stay out of the duration sampler, which reports the
    // variant that runs afterwards
    const bool prof_on = c.prof_on;
    c.prof_on = false;
    hipEvent_t ev[2];
    HIPCHK(hipEventCreate(&ev[0]));
    HIPCHK(hipEventCreate(&ev[1]));
    float best = 0.0f;
    int pick = 0;
    for (int v = 0; v < 4; ++v) {
        if (!reg_variant_ok(c, v)) continue;
        const int lay = v;
        set_reg_variant(c, v);
        reg_k(c, x, y, c.freem, 1, st);
        HIPCHK(hipEventRecord(ev[0], st));
        for (int r = 0; r < 5; ++r) reg_k(c, x, y, c.freem, 1, st);
        HIPCHK(hipEventRecord(ev[1], st));
        HIPCHK(hipEventSynchronize(ev[1]));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
        c.tune_ms[lay] = ms / 5.0f;
        if (best == 0.0f || ms < best) {
            best = ms;
            pick = lay;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    c.prof_on = prof_on;
    set_reg_variant(c, pick);
    if (log_enabled())
        fprintf(stderr, "[fcrkpm] register variants (8 lanes, 16 lanes; x2 tiles): %.1f %.1f %.1f %.1f us;"
                " using %d\n", 1e3 * c.tune_ms[0], 1e3 * c.tune_ms[1], 1e3 * c.tune_ms[2],
                1e3 * c.tune_ms[3], pick);
}

// Lines per workgroup of the LDS-tiled passes (16, 8 or 4), chosen by timing
// K products of each precision that runs on them (not where the register path
// serves that precision).
void tune_sep_tiles(Ctx& c, hipStream_t st)
{
    const bool need[2] = {!use_reg_path(c, 1), !use_reg_path64(c)};
    if (!need[0] && !need[1]) return;
    const bool prof_on = c.prof_on;
    c.prof_on = false;
    hipEvent_t ev[2];
    HIPCHK(hipEventCreate(&ev[0]));
    HIPCHK(hipEventCreate(&ev[1]));
    double* x64 = vec64(c, V_T);
    double* y64 = vec64(c, V_Q);
    float* x32 = vec32(c, 2);
    float* y32 = vec32(c, 3);
    HIPCHK(hipMemsetAsync(x64, 0, sizeof(double) * c.nn, st));
    HIPCHK(hipMemsetAsync(x32, 0, sizeof(float) * c.nn, st));
    static const int caps[3] = {16, 8, 4};
    for (int pr = 0; pr < 2; ++pr) {
        if (!need[pr]) continue;
        float best = 0.0f;
        int pick = 16;
        for (int cap : caps) {
            c.sep_wcap[pr] = cap;
            auto one = [&]() {
                if (pr == 0) apply_one<float>(c, FCRKPM_OP_K, x32, y32, 1, st);
                else apply_one<double>(c, FCRKPM_OP_K, x64, y64, 1, st);
            };
            one();
            HIPCHK(hipEventRecord(ev[0], st));
            for (int r = 0; r < 3; ++r) one();
            HIPCHK(hipEventRecord(ev[1], st));
            HIPCHK(hipEventSynchronize(ev[1]));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
            if (best == 0.0f || ms < best) {
                best = ms;
                pick = cap;
            }
        }
        c.sep_wcap[pr] = pick;
        if (log_enabled())
            fprintf(stderr, "[fcrkpm] LDS-tiled %s K product: %d lines per workgroup (%.1f us)\n",
                    pr ? "FP64" : "FP32", pick, 1e3 * best / 3.0f);
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    c.prof_on = prof_on;
}

// The autotuner's key for this device and problem shape, "" without a cache
std::string tune_key(const Ctx& c)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "";
    }
    char buf[256];
    snprintf(buf, sizeof(buf), "%s/%dcu/n%dx%dx%d/d%d/deg%d/m%d.%d.%d/lc%d", prop.gcnArchName,
             prop.multiProcessorCount, c.n[0], c.n[1], c.n[2], c.dim, c.degree, c.m[0], c.m[1], c.m[2],
             (c.use_sym && c.sym) ? 1 : 0);
    return buf;
}

// Setup-time autotuner: the register path's line layout and tiles per
// workgroup, and the LDS-tiled passes' lines per workgroup.  With
// FCRKPM_AUTOTUNE_CACHE naming a file, choices are looked up there by device
// and problem shape (no timing on a hit) and new ones appended, one line each:
// "<key> <register variant> <FP32 lines> <FP64 lines> <4 variant times, us>".
void autotune(Ctx& c, hipStream_t st)
{
    const char* path = getenv("FCRKPM_AUTOTUNE_CACHE");
    const std::string key = (path && *path) ? tune_key(c) : std::string();
    if (!key.empty()) {
        if (FILE* f = fopen(path, "r")) {
            char line[512];
            bool hit = false;
            int v = 0, w32 = 16, w64 = 16;
            float t[4] = {};
            while (fgets(line, sizeof(line), f)) {
                char k[256];
                int vv, a32, a64;
                float tt[4];
                if (sscanf(line, "%255s %d %d %d %f %f %f %f", k, &vv, &a32, &a64, &tt[0], &tt[1], &tt[2],
                           &tt[3]) == 8 &&
                    key == k) {
                    hit = true;
                    v = vv;
                    w32 = a32;
                    w64 = a64;
                    for (int i = 0; i < 4; ++i) t[i] = tt[i];
                }
            }
            fclose(f);
            const bool ok_caps = (w32 == 16 || w32 == 8 || w32 == 4) && (w64 == 16 || w64 == 8 || w64 == 4);
            const bool ok_var = !(reg_path_ok(c) || reg_gpq_ok(c)) || reg_variant_ok(c, v);
            if (hit && ok_caps && ok_var) {
                if (reg_path_ok(c) || reg_gpq_ok(c)) set_reg_variant(c, v);
                c.sep_wcap[0] = w32;
                c.sep_wcap[1] = w64;
                for (int i = 0; i < 4; ++i) c.tune_ms[i] = t[i] * 1e-3f;
                c.tune_cached = true;
                if (log_enabled()) fprintf(stderr, "[fcrkpm] autotune cache hit: %s\n", key.c_str());
                return;
            }
        }
    }
    if (const char* e = getenv("FCRKPM_REGLAYOUT")) {
        if (*e >= '0' && *e <= '3' && reg_variant_ok(c, *e - '0')) {
            set_reg_variant(c, *e - '0');
            tune_sep_tiles(c, st);
            return;
        }
    }
    tune_reg_layout(c, st);
    tune_sep_tiles(c, st);
    if (!key.empty()) {
        if (FILE* f = fopen(path, "a")) {
            fprintf(f, "%s %d %d %d %.3f %.3f %.3f %.3f\n", key.c_str(), c.reg_layout + 2 * (c.reg_tpw - 1),
                    c.sep_wcap[0], c.sep_wcap[1], 1e3f * c.tune_ms[0], 1e3f * c.tune_ms[1], 1e3f * c.tune_ms[2],
                    1e3f * c.tune_ms[3]);
            fclose(f);
        }
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
        if (degree < 1 || degree > 3 || (degree == 3 && grid->dim == 3))
            fail(FCRKPM_ERR_ARG, "degree must be 1 or 2, or 3 in 1D and 2D");
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
                if (!make_plan(c.n[a], c.plan[a])) fail(FCRKPM_ERR_ARG, "box size must factor into 2, 3, 5 and 7");
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

        // the static scratch of fcrkpm_apply_noalloc on this device
        c.scratch = scratch_address();

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
            {
                // t_e is even or odd in the offset with e, so T_e is real or
                // imaginary: the register passes take Re T_0, Im T_1, Re T_2,
                // each with the 1/L of the inverse transform folded in
                std::vector<float> rt((size_t)3 * L, 0.0f);
                for (int e = 0; e < 3 && e < ne; ++e)
                    for (int kk = 0; kk < L; ++kk)
                        rt[(size_t)e * L + kk] = (float)(((e & 1) ? sp[(size_t)e * L + kk].y
                                                                  : sp[(size_t)e * L + kk].x) / L);
                c.rtab32[a] = dalloc<float>(rt.size());
                HIPCHK(hipMemcpyAsync(c.rtab32[a], rt.data(), sizeof(float) * rt.size(),
                                      hipMemcpyHostToDevice, st));
                std::vector<double> rt64((size_t)3 * L, 0.0);
                for (int e = 0; e < 3 && e < ne; ++e)
                    for (int kk = 0; kk < L; ++kk)
                        rt64[(size_t)e * L + kk] = ((e & 1) ? sp[(size_t)e * L + kk].y
                                                            : sp[(size_t)e * L + kk].x) / L;
                c.rtab64[a] = dalloc<double>(rt64.size());
                HIPCHK(hipMemcpyAsync(c.rtab64[a], rt64.data(), sizeof(double) * rt64.size(),
                                      hipMemcpyHostToDevice, st));
                HIPCHK(hipStreamSynchronize(st));
            }
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

        c.krows = c.dim;
        build_pointwise(c, st);
        if (const char* e = getenv("FCRKPM_SYM")) c.use_sym = *e != '0';
        sym_build(c, st);
        // the FP64 register path's records of u^h, f^r and the gradient force,
        // built here so that no later product allocates them
        (void)reg_kn_ok(c, st);

        // workspace and solver buffers for one right-hand side; both grow on demand
        HIPCHK(hipStreamSynchronize(st));
        ensure_work(c, 1);
        ensure_rhs(c, 1);
        autotune(c, st);
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

namespace {
// b = chi_Omega (f^r + f^q - K d_Gamma) and x = chi_Omega d0 for nrhs fields
// (Eq 28-29, Alg 5, Alg A.1; f^q only with a flux q)
void prepare_solve(Ctx& c, int nrhs, const double* r, const double* g, const double* d0,
                   hipStream_t st, const double* qflux = nullptr)
{
    ensure_rhs(c, nrhs);
    ensure_work(c, nrhs);
    const long nn = c.nn;
    HIPCHK(hipMemsetAsync(c.dflag + 2, 0, sizeof(int), st));
    launch_check_finite(r, nn * nrhs, c.dflag + 2, st);
    if (g) launch_check_finite(g, nn * nrhs, c.dflag + 2, st);
    if (d0) launch_check_finite(d0, nn * nrhs, c.dflag + 2, st);
    if (qflux) launch_check_finite(qflux, nn * nrhs, c.dflag + 2, st);
    int hf = 0;
    HIPCHK(hipMemcpyAsync(&hf, c.dflag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hf) fail(FCRKPM_ERR_ARG, "non-finite value in r, q, g or the initial guess");
    double* b = vec64(c, V_B);
    double* x = vec64(c, V_X);
    double* t = vec64(c, V_T);
    double* p = vec64(c, V_P);
    double* q = vec64(c, V_Q);
    apply_one<double>(c, FCRKPM_OP_FR, r, t, nrhs, st);  // f^r (Alg 4)
    if (qflux) {
        apply_one<double>(c, FCRKPM_OP_FQ, qflux, q, nrhs, st);  // f^q (Alg A.1)
        launch_lincomb_masked(t, 1.0, q, 1.0, nullptr, c.chi, t, nn, nrhs, st);
    }
    if (g) {
        launch_masked_copy<double>(g, c.dirm, p, nn, nrhs, st);  // d_Gamma
        apply_one<double>(c, FCRKPM_OP_K_FULL, p, q, nrhs, st);
        launch_sub_masked(t, q, c.freem, b, nn, nrhs, st);
    } else {
        launch_masked_copy<double>(t, c.freem, b, nn, nrhs, st);
    }
    if (d0) launch_masked_copy<double>(d0, c.freem, x, nn, nrhs, st);
    else HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * nn * nrhs, st));
}

// d = chi_Omega x + chi_Gamma_g g, and u^h = N d when asked (Alg 3)
void finish_solve(Ctx& c, int nrhs, const double* g, double* d_out, double* uh_out,
                  hipStream_t st)
{
    const long nn = c.nn;
    double* x = vec64(c, V_X);
    if (g) {
        double* p = vec64(c, V_P);
        launch_masked_copy<double>(g, c.dirm, p, nn, nrhs, st);
        launch_select(c.freem, x, p, d_out, nn, nrhs, st);
    } else {
        HIPCHK(hipMemcpyAsync(d_out, x, sizeof(double) * nn * nrhs, hipMemcpyDeviceToDevice, st));
    }
    if (uh_out) apply_one<double>(c, FCRKPM_OP_UH, d_out, uh_out, nrhs, st);
}

void check_solve_args(int mode, int nrhs, double tol, int maxit)
{
    if (mode < FCRKPM_MODE_F64 || mode > FCRKPM_MODE_F32_PRODUCTS) fail(FCRKPM_ERR_ARG, "unknown mode");
    if (nrhs < 1 || nrhs > 65535) fail(FCRKPM_ERR_ARG, "nrhs must be in [1, 65535]");
    if (!(tol > 0.0) || maxit < 1) fail(FCRKPM_ERR_ARG, "tol must be > 0 and maxit >= 1");
}
}  // namespace

extern "C" fcrkpm_status fcrkpm_apply(fcrkpm_ctx* ctx, int32_t op, int32_t dtype, int32_t nrhs,
                                      const void* in, void* out, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (op < FCRKPM_OP_K || op > FCRKPM_OP_FQ) fail(FCRKPM_ERR_ARG, "unknown operator");
        if (dtype != FCRKPM_F64 && dtype != FCRKPM_F32) fail(FCRKPM_ERR_ARG, "unknown dtype");
        if (nrhs < 1 || nrhs > 65535) fail(FCRKPM_ERR_ARG, "nrhs must be in [1, 65535]");
        if (!in || !out) fail(FCRKPM_ERR_ARG, "NULL array");
        const size_t es = dtype == FCRKPM_F64 ? 8 : 4;
        const char* a0 = (const char*)in;
        const char* b0 = (const char*)out;
        const size_t bytes = es * (size_t)c.nn * nrhs;
        if (a0 < b0 + bytes && b0 < a0 + bytes) fail(FCRKPM_ERR_ARG, "in and out overlap");
        hipStream_t st = (hipStream_t)stream;
        if (dtype == FCRKPM_F64)
            apply_one<double>(c, op, (const double*)in, (double*)out, nrhs, st);
        else
            apply_one<float>(c, op, (const float*)in, (float*)out, nrhs, st);
        HIPCHK(hipGetLastError());
        return FCRKPM_OK;
    });
}

extern "C" fcrkpm_status fcrkpm_apply_noalloc(fcrkpm_ctx* ctx, int32_t op, int32_t dtype, int32_t nrhs,
                                              const void* in, void* out, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (op < FCRKPM_OP_K || op > FCRKPM_OP_FQ) fail(FCRKPM_ERR_ARG, "unknown operator");
        if (dtype != FCRKPM_F64 && dtype != FCRKPM_F32) fail(FCRKPM_ERR_ARG, "unknown dtype");
        if (nrhs < 1 || nrhs > 65535) fail(FCRKPM_ERR_ARG, "nrhs must be in [1, 65535]");
        if (!in || !out) fail(FCRKPM_ERR_ARG, "NULL array");
        // the first FCRKPM_OP_M product builds the mass coefficients, which allocates
        if (op == FCRKPM_OP_M && !c.mass_set)
            fail(FCRKPM_ERR_ARG, "the consistent mass is not built yet: call fcrkpm_apply with "
                                 "FCRKPM_OP_M once first");
        if (!c.scratch) fail(FCRKPM_ERR_ARG, "context has no scratch address");
        const size_t es = dtype == FCRKPM_F64 ? 8 : 4;
        const char* a0 = (const char*)in;
        const char* b0 = (const char*)out;
        const size_t bytes = es * (size_t)c.nn * nrhs;
        if (a0 < b0 + bytes && b0 < a0 + bytes) fail(FCRKPM_ERR_ARG, "in and out overlap");
        // two workspace slots of maxpairs complex fields per right-hand side
        const size_t need = (size_t)2 * c.basis_plan.maxpairs * c.nn * nrhs * (2 * es);
        if (need > kScratchBytes)
            fail(FCRKPM_ERR_ARG, "the product needs " + std::to_string(need) +
                                     " bytes of scratch; the static scratch holds " +
                                     std::to_string(kScratchBytes));
        // the passes take their workspace from the context: point it at the
        // scratch for this call (no kernel reads a workspace value it has not
        // written in the same call, so nothing needs clearing) and put the
        // context's own workspace back afterwards
        struct WorkSwap {
            Ctx& c;
            cplx<float>* w32;
            cplx<double>* w64;
            int cap;
            WorkSwap(Ctx& c_, int nrhs) : c(c_), w32(c_.work32), w64(c_.work64), cap(c_.cap_work)
            {
                c.work32 = reinterpret_cast<cplx<float>*>(c.scratch);
                c.work64 = reinterpret_cast<cplx<double>*>(c.scratch);
                c.cap_work = nrhs;
            }
            ~WorkSwap()
            {
                c.work32 = w32;
                c.work64 = w64;
                c.cap_work = cap;
            }
        } swap(c, nrhs);
        hipStream_t st = (hipStream_t)stream;
        if (dtype == FCRKPM_F64)
            apply_one<double>(c, op, (const double*)in, (double*)out, nrhs, st);
        else
            apply_one<float>(c, op, (const float*)in, (float*)out, nrhs, st);
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
        check_solve_args(mode, nrhs, tol, maxit);
        if (!r || !d_inout) fail(FCRKPM_ERR_ARG, "NULL array");
        hipStream_t st = (hipStream_t)stream;
        prepare_solve(c, nrhs, r, g, d_inout, st);
        Solver S(c, nrhs, mode, tol, maxit);
        run_solvers({&S}, graphs_enabled(c), st);
        const fcrkpm_status worst = S.finish(info, st);
        finish_solve(c, nrhs, g, d_inout, uh_out, st);
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (worst != FCRKPM_OK) c.err = "solver did not reach the tolerance";
        return worst;
    });
}

extern "C" fcrkpm_status fcrkpm_solve_flux(fcrkpm_ctx* ctx, int32_t mode, int32_t nrhs,
                                           const double* r, const double* q, const double* g,
                                           double* d_inout, double* uh_out, double tol,
                                           int32_t maxit, fcrkpm_info* info, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        check_solve_args(mode, nrhs, tol, maxit);
        if (!r || !q || !d_inout) fail(FCRKPM_ERR_ARG, "NULL array");
        if (!c.area64) fail(FCRKPM_ERR_ARG, "no boundary areas: call fcrkpm_set_boundary first");
        hipStream_t st = (hipStream_t)stream;
        prepare_solve(c, nrhs, r, g, d_inout, st, q);
        Solver S(c, nrhs, mode, tol, maxit);
        run_solvers({&S}, graphs_enabled(c), st);
        const fcrkpm_status worst = S.finish(info, st);
        finish_solve(c, nrhs, g, d_inout, uh_out, st);
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (worst != FCRKPM_OK) c.err = "solver did not reach the tolerance";
        return worst;
    });
}

extern "C" fcrkpm_status fcrkpm_set_boundary(fcrkpm_ctx* ctx, const double* area, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        hipStream_t st = (hipStream_t)stream;
        HIPCHK(hipStreamSynchronize(st));
        dfree(c.area64);
        dfree(c.area32);
        if (!area) return FCRKPM_OK;
        HIPCHK(hipMemsetAsync(c.dflag + 2, 0, sizeof(int), st));
        launch_check_finite(area, c.nn, c.dflag + 2, st);
        int hf = 0;
        HIPCHK(hipMemcpyAsync(&hf, c.dflag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hf) fail(FCRKPM_ERR_ARG, "non-finite boundary area");
        c.area64 = dalloc<double>(c.nn);
        c.area32 = dalloc<float>(c.nn);
        HIPCHK(hipMemcpyAsync(c.area64, area, sizeof(double) * c.nn, hipMemcpyDeviceToDevice, st));
        launch_to32(c.area64, c.area32, c.nn, st);
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        return FCRKPM_OK;
    });
}

extern "C" fcrkpm_status fcrkpm_solve_batch(fcrkpm_ctx* const* ctxs, int32_t nprob, int32_t mode,
                                            const int32_t* nrhs, const double* const* r,
                                            const double* const* g, double* const* d_inout,
                                            double* const* uh_out, double tol, int32_t maxit,
                                            fcrkpm_info* info, void* stream)
{
    if (!ctxs || nprob < 1 || !ctxs[0]) {
        g_setup_err = "fcrkpm_solve_batch: no problems";
        return FCRKPM_ERR_ARG;
    }
    std::string err;
    fcrkpm_status s = run_guarded(err, [&]() -> fcrkpm_status {
        if (!nrhs || !r || !d_inout) fail(FCRKPM_ERR_ARG, "NULL array");
        for (int p = 0; p < nprob; ++p) {
            if (!ctxs[p]) fail(FCRKPM_ERR_ARG, "NULL context in the batch");
            for (int q = 0; q < p; ++q)
                if (ctxs[q] == ctxs[p]) fail(FCRKPM_ERR_ARG, "a context appears twice in the batch");
            check_solve_args(mode, nrhs[p], tol, maxit);
            if (!r[p] || !d_inout[p]) fail(FCRKPM_ERR_ARG, "NULL array in the batch");
        }
        hipStream_t st = (hipStream_t)stream;
        bool graphs = true;
        for (int p = 0; p < nprob; ++p) {
            Ctx& c = ctxs[p]->c;
            prepare_solve(c, nrhs[p], r[p], g ? g[p] : nullptr, d_inout[p], st);
            graphs = graphs && graphs_enabled(c);
        }
        std::vector<std::unique_ptr<Solver>> S;
        std::vector<Solver*> ptr;
        for (int p = 0; p < nprob; ++p) {
            S.emplace_back(new Solver(ctxs[p]->c, nrhs[p], mode, tol, maxit));
            ptr.push_back(S.back().get());
        }
        run_solvers(ptr, graphs, st);
        fcrkpm_status worst = FCRKPM_OK;
        long off = 0;
        for (int p = 0; p < nprob; ++p) {
            const fcrkpm_status sp = S[p]->finish(info ? info + off : nullptr, st);
            if (sp != FCRKPM_OK) worst = sp;
            off += nrhs[p];
        }
        for (int p = 0; p < nprob; ++p)
            finish_solve(ctxs[p]->c, nrhs[p], g ? g[p] : nullptr, d_inout[p],
                         uh_out ? uh_out[p] : nullptr, st);
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (worst != FCRKPM_OK) err = "a problem of the batch did not reach the tolerance";
        return worst;
    });
    for (int p = 0; p < nprob; ++p)
        if (ctxs[p]) ctxs[p]->c.err = err;
    return s;
}

extern "C" fcrkpm_status fcrkpm_adjoint(fcrkpm_ctx* ctx, int32_t mode, int32_t nrhs,
                                        const double* dl_duh, double* dl_dr, double tol,
                                        int32_t maxit, fcrkpm_info* info, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        check_solve_args(mode, nrhs, tol, maxit);
        if (!dl_duh || !dl_dr) fail(FCRKPM_ERR_ARG, "NULL array");
        hipStream_t st = (hipStream_t)stream;
        ensure_rhs(c, nrhs);
        ensure_work(c, nrhs);
        const long nn = c.nn;
        double* b = vec64(c, V_B);
        double* x = vec64(c, V_X);
        double* t = vec64(c, V_T);
        apply_one<double>(c, FCRKPM_OP_NT, dl_duh, t, nrhs, st);
        launch_masked_copy<double>(t, c.freem, b, nn, nrhs, st);
        HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * nn * nrhs, st));
        Solver S(c, nrhs, mode, tol, maxit);
        run_solvers({&S}, graphs_enabled(c), st);
        const fcrkpm_status worst = S.finish(info, st);
        apply_one<double>(c, FCRKPM_OP_VN, x, dl_dr, nrhs, st);
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (worst != FCRKPM_OK) c.err = "adjoint solve did not reach the tolerance";
        return worst;
    });
}

// Time stepping of the diffusion problem M d' + nu K d = f^r (App. C, Eq C.1-
// C.4) with d = g held on the Dirichlet nodes and r constant in time.  On the
// free rows, with x the free part of d and c0 = dt (f^r - nu K d_Gamma):
//   implicit (Alg C.4): (M + theta dt nu K) x1 = (M - (1-theta) dt nu K) x0 + c0,
//     one CG solve per step (the solver of fcrkpm_solve on the shifted
//     operator, warm-started from x0);
//   explicit (Alg C.3): x1 = x0 + (c0 - dt nu K x0) / M^l.
extern "C" fcrkpm_status fcrkpm_transient(fcrkpm_ctx* ctx, const fcrkpm_time* tp, int32_t mode,
                                          int32_t nrhs, const double* r, const double* g,
                                          double* d_inout, double* uh_out, double tol,
                                          int32_t maxit, fcrkpm_info* info, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (!tp || !d_inout) fail(FCRKPM_ERR_ARG, "NULL argument");
        const fcrkpm_time T = *tp;
        const bool implicit = T.scheme == FCRKPM_TIME_IMPLICIT;
        if (!implicit && T.scheme != FCRKPM_TIME_EXPLICIT_LUMPED) fail(FCRKPM_ERR_ARG, "unknown time scheme");
        if (T.nsteps < 0) fail(FCRKPM_ERR_ARG, "nsteps must be >= 0");
        if (!(T.dt > 0.0) || !std::isfinite(T.dt) || !(T.nu > 0.0) || !std::isfinite(T.nu))
            fail(FCRKPM_ERR_ARG, "dt and nu must be finite and > 0");
        if (implicit && !(T.theta > 0.0 && T.theta <= 1.0)) fail(FCRKPM_ERR_ARG, "theta must be in (0, 1]");
        check_solve_args(mode, nrhs, tol, maxit);
        if (!implicit && mode != FCRKPM_MODE_F64)
            fail(FCRKPM_ERR_UNSUPPORTED, "the explicit scheme runs FP64 products only");
        hipStream_t st = (hipStream_t)stream;
        const long nn = c.nn;
        ensure_rhs(c, nrhs);
        ensure_work(c, nrhs);
        HIPCHK(hipMemsetAsync(c.dflag + 2, 0, sizeof(int), st));
        if (r) launch_check_finite(r, nn * nrhs, c.dflag + 2, st);
        if (g) launch_check_finite(g, nn * nrhs, c.dflag + 2, st);
        launch_check_finite(d_inout, nn * nrhs, c.dflag + 2, st);
        int hf = 0;
        HIPCHK(hipMemcpyAsync(&hf, c.dflag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hf) fail(FCRKPM_ERR_ARG, "non-finite value in r, g or d");

        struct Buf {
            double* p = nullptr;
            ~Buf() { dfree(p); }
        } c0b;
        c0b.p = dalloc<double>((size_t)nn * nrhs);
        double* c0 = c0b.p;
        double* x = vec64(c, V_X);
        double* t = vec64(c, V_T);
        double* q = vec64(c, V_Q);
        double* pv = vec64(c, V_P);
        if (r) apply_one<double>(c, FCRKPM_OP_FR, r, t, nrhs, st);  // f^r (Alg 4)
        else HIPCHK(hipMemsetAsync(t, 0, sizeof(double) * nn * nrhs, st));
        if (g) {
            launch_masked_copy<double>(g, c.dirm, pv, nn, nrhs, st);  // d_Gamma
            apply_one<double>(c, FCRKPM_OP_K_FULL, pv, q, nrhs, st);
            launch_lincomb_masked(t, T.dt, q, -T.dt * T.nu, nullptr, c.freem, c0, nn, nrhs, st);
        } else {
            launch_lincomb_masked(t, T.dt, nullptr, 0.0, nullptr, c.freem, c0, nn, nrhs, st);
        }
        launch_masked_copy<double>(d_inout, c.freem, x, nn, nrhs, st);

        std::vector<fcrkpm_info> acc(nrhs);
        memset(acc.data(), 0, sizeof(fcrkpm_info) * nrhs);
        fcrkpm_status worst = FCRKPM_OK;
        if (implicit) {
            OpSet* ms = mass_set(c, st);
            OpSet* as = shift_set(c, 1.0, T.theta * T.dt * T.nu, st);
            std::vector<fcrkpm_info> inf(nrhs);
            for (int step = 0; step < T.nsteps && worst == FCRKPM_OK; ++step) {
                double* b = vec64(c, V_B);
                {
                    SetScope use(c, ms);
                    apply_one<double>(c, FCRKPM_OP_K, x, t, nrhs, st);  // M x0 (Alg C.1)
                }
                if (T.theta < 1.0) {
                    apply_one<double>(c, FCRKPM_OP_K, x, q, nrhs, st);
                    launch_lincomb_masked(t, 1.0, q, -(1.0 - T.theta) * T.dt * T.nu, c0, c.freem, b,
                                          nn, nrhs, st);
                } else {
                    launch_lincomb_masked(t, 1.0, nullptr, 0.0, c0, c.freem, b, nn, nrhs, st);
                }
                SetScope use(c, as);
                Solver S(c, nrhs, mode, tol, maxit);
                run_solvers({&S}, graphs_enabled(c), st);
                worst = S.finish(inf.data(), st);
                for (int j = 0; j < nrhs; ++j) {
                    fcrkpm_info& a = acc[j];
                    const fcrkpm_info& f = inf[j];
                    a.iters += f.iters;
                    a.outer_iters += f.outer_iters;
                    a.rel_res = std::max(a.rel_res, f.rel_res);
                    a.true_rel_res = std::max(a.true_rel_res, f.true_rel_res);
                    a.fallback_used |= f.fallback_used;
                    a.matvecs_f64 += f.matvecs_f64 + (T.theta < 1.0 ? 2 : 1);
                    a.matvecs_f32 += f.matvecs_f32;
                }
            }
        } else {
            // M^l (Eq C.13, Alg C.2) in the first field of V_R
            double* ml = vec64(c, V_R);
            launch_mask_to_double(c.chi, q, nn, st);
            apply_one<double>(c, FCRKPM_OP_FR, q, ml, 1, st);
            HIPCHK(hipMemsetAsync(c.dflag + 2, 0, sizeof(int), st));
            launch_check_positive(ml, c.freem, nn, c.dflag + 2, st);
            HIPCHK(hipMemcpyAsync(&hf, c.dflag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (hf) fail(FCRKPM_ERR_SINGULAR, "lumped mass not positive on a free node");
            for (int step = 0; step < T.nsteps; ++step) {
                apply_one<double>(c, FCRKPM_OP_K, x, t, nrhs, st);
                launch_explicit_update(x, t, c0, ml, T.dt * T.nu, c.freem, nn, nrhs, st);
            }
            for (auto& a : acc) a.matvecs_f64 = T.nsteps;
        }
        finish_solve(c, nrhs, g, d_inout, uh_out, st);
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (info) memcpy(info, acc.data(), sizeof(fcrkpm_info) * nrhs);
        if (worst != FCRKPM_OK) c.err = "a time step's solve did not reach the tolerance";
        return worst;
    });
}

// The nonlinear force of N(u) = kappa u^3 (App. B, Eq B.2, B.9; Alg B.2):
// u^h = N d (Alg 3), the pointwise nonlinearity, then the load pass (Alg 4).
extern "C" fcrkpm_status fcrkpm_nonlinear_force(fcrkpm_ctx* ctx, double kappa, int32_t nrhs,
                                                const double* d, double* out, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (!d || !out) fail(FCRKPM_ERR_ARG, "NULL array");
        if (nrhs < 1 || nrhs > 65535) fail(FCRKPM_ERR_ARG, "nrhs must be in [1, 65535]");
        if (!std::isfinite(kappa)) fail(FCRKPM_ERR_ARG, "kappa must be finite");
        hipStream_t st = (hipStream_t)stream;
        ensure_rhs(c, nrhs);
        ensure_work(c, nrhs);
        double* u = vec64(c, V_T);
        apply_one<double>(c, FCRKPM_OP_UH, d, u, nrhs, st);
        launch_pow_scaled(u, kappa, 3, u, c.nn * nrhs, st);
        apply_one<double>(c, FCRKPM_OP_FR, u, out, nrhs, st);
        HIPCHK(hipGetLastError());
        return FCRKPM_OK;
    });
}

// Force of the gradient nonlinearity N(grad u) = (1 + kappa |grad u|^2) grad u
// (App. B, Eq B.5-B.8, B.10; Alg B.1): the passes of K with the nonlinearity
// applied to the implicit gradient A^a = sum_q b^a_q D_q before E_p is formed.
extern "C" fcrkpm_status fcrkpm_gradient_force(fcrkpm_ctx* ctx, double kappa, int32_t nrhs,
                                               const double* d, double* out, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (!d || !out) fail(FCRKPM_ERR_ARG, "NULL array");
        if (nrhs < 1 || nrhs > 65535) fail(FCRKPM_ERR_ARG, "nrhs must be in [1, 65535]");
        if (!std::isfinite(kappa)) fail(FCRKPM_ERR_ARG, "kappa must be finite");
        const size_t bytes = sizeof(double) * (size_t)c.nn * nrhs;
        if ((const char*)d < (const char*)out + bytes && (const char*)out < (const char*)d + bytes)
            fail(FCRKPM_ERR_ARG, "d and out overlap");
        c.pw_kappa = kappa;
        apply_one<double>(c, OP_KN, d, out, nrhs, (hipStream_t)stream);
        HIPCHK(hipGetLastError());
        return FCRKPM_OK;
    });
}

namespace {
// B x: the implicit gradient at every node, component a from the u^h passes
// with the coefficient rows b^a in place of b^0 (Eq 15-16, Alg 3 with b^a)
void apply_grad(Ctx& c, const double* x, double* out, hipStream_t st)
{
    if (use_reg_path64(c) && reg_kn_ok(c, st)) {
        launch_reg_kn(c, x, out, 0.0, RK_GRAD, st);
        return;
    }
    double* keep = c.b0_64;
    struct Restore {
        Ctx& c;
        double* p;
        ~Restore() { c.b0_64 = p; }
    } restore{c, keep};
    for (int a = 0; a < c.dim; ++a) {
        c.b0_64 = c.ba_64 + (size_t)a * c.s * c.nn;
        apply_one<double>(c, FCRKPM_OP_UH, x, out + (size_t)a * c.nn, 1, st);
    }
}
}  // namespace

// Alg B.3: the static nonlinear problem by nonlinear conjugate gradients.  The
// forces of App. B (Eq B.2/B.4 with N(u) = kappa u^3, Eq B.6/B.8 with N(g) =
// (1 + kappa |g|^2) g) are the gradients of convex energies, so the residual
// R(d) is driven to zero by minimising along conjugate directions
// (Polak-Ribiere, restarted when beta < 0) with an exact line search: phi'(alpha)
// = R(d + alpha p) . p is a linear part plus nodal sums in u + alpha w or
// g + alpha h (w = N p, h = B p), and Newton's method on it needs one
// reduction kernel per step and no transform.  Every iteration costs one
// force evaluation and the products of p (K p and N p, or B p).
extern "C" fcrkpm_status fcrkpm_solve_nonlinear_cg(fcrkpm_ctx* ctx, int32_t kind, double kappa,
                                                   const double* r, const double* g, double* d_inout,
                                                   double* uh_out, double tol, int32_t maxit,
                                                   fcrkpm_info* info, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    std::vector<double*> bufs;
    struct Free {
        std::vector<double*>& b;
        ~Free()
        {
            for (double*& p : b) dfree(p);
        }
    } release_bufs{bufs};
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (kind != FCRKPM_NONLIN_CUBIC && kind != FCRKPM_NONLIN_GRADIENT) fail(FCRKPM_ERR_ARG, "unknown nonlinearity");
        if (!r || !d_inout) fail(FCRKPM_ERR_ARG, "NULL array");
        if (!(kappa >= 0.0) || !std::isfinite(kappa)) fail(FCRKPM_ERR_ARG, "kappa must be finite and >= 0");
        if (!(tol > 0.0) || maxit < 1) fail(FCRKPM_ERR_ARG, "tol must be > 0 and maxit >= 1");
        hipStream_t st = (hipStream_t)stream;
        const long nn = c.nn;
        const int dim = c.dim;
        ensure_rhs(c, 1);
        ensure_work(c, 1);
        HIPCHK(hipMemsetAsync(c.dflag + 2, 0, sizeof(int), st));
        launch_check_finite(r, nn, c.dflag + 2, st);
        if (g) launch_check_finite(g, nn, c.dflag + 2, st);
        launch_check_finite(d_inout, nn, c.dflag + 2, st);
        int hf = 0;
        HIPCHK(hipMemcpyAsync(&hf, c.dflag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hf) fail(FCRKPM_ERR_ARG, "non-finite value in r, g or d");
        auto vec = [&](int count) {
            double* p = dalloc<double>((size_t)count * nn);
            bufs.push_back(p);
            return p;
        };
        const bool cubic = kind == FCRKPM_NONLIN_CUBIC;
        double* d = vec(1);
        double* fr = vec(1);
        double* R = vec(1);
        double* rr = vec(1);
        double* p = vec(1);
        double* t = vec(1);
        double* ro = vec(1);                 // the previous residual
        double* a = vec(cubic ? 1 : dim);   // u = N d, or g = B d
        double* b = vec(cubic ? 1 : dim);   // w = N p, or h = B p
        double* kd = cubic ? vec(1) : nullptr;
        double* kp = cubic ? vec(1) : nullptr;
        // the line search's partials (4 x kRedBlocks) and its 4 sums (kScal apart)
        double* lsb = dalloc<double>(4 * (size_t)kRedBlocks + 4 * (size_t)kScal);
        bufs.push_back(lsb);
        std::vector<double> hq(4 * (size_t)kScal);
        int products = 0;

        // d: g on the Dirichlet nodes, the initial guess on the free nodes
        launch_lincomb_masked(d_inout, 1.0, nullptr, 0.0, nullptr, c.freem, d, nn, 1, st);
        if (g) {
            launch_lincomb_masked(g, 1.0, nullptr, 0.0, nullptr, c.dirm, t, nn, 1, st);
            launch_lincomb_masked(d, 1.0, t, 1.0, nullptr, c.chi, d, nn, 1, st);
        }
        apply_one<double>(c, FCRKPM_OP_FR, r, fr, 1, st);
        launch_lincomb_masked(fr, 1.0, nullptr, 0.0, nullptr, c.freem, t, nn, 1, st);
        dots<double>(c, t, t, 1, S_BB, st);
        const double fnorm = sqrt(read_scalars(c, 1, st)[S_BB]);
        if (cubic) {
            apply_one<double>(c, FCRKPM_OP_UH, d, a, 1, st);
            apply_one<double>(c, FCRKPM_OP_K_FULL, d, kd, 1, st);
            ++products;
        } else {
            apply_grad(c, d, a, st);
        }
        // rr = -R(d) on the free rows
        auto residual = [&]() {
            if (cubic) {
                launch_pow_scaled(a, kappa, 3, t, nn, st);
                apply_one<double>(c, FCRKPM_OP_FR, t, R, 1, st);
                launch_lincomb_masked(kd, 1.0, R, 1.0, nullptr, c.freem, R, nn, 1, st);
            } else {
                c.pw_kappa = kappa;
                apply_one<double>(c, OP_KN, d, R, 1, st);
                ++products;
            }
            launch_lincomb_masked(fr, 1.0, R, -1.0, nullptr, c.freem, rr, nn, 1, st);
        };
        residual();
        HIPCHK(hipMemcpyAsync(p, rr, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
        dots<double>(c, rr, rr, 1, S_NORM, st);
        double rn = read_scalars(c, 1, st)[S_NORM];
        int it = 0, lsteps = 0;
        bool conv = fnorm == 0.0;
        const double* vol = c.vol64;
        while (!conv && it < maxit) {
            if (sqrt(rn) <= tol * fnorm) {
                conv = true;
                break;
            }
            // exact line search along p
            double c0, c1 = 0.0;
            if (cubic) {
                apply_one<double>(c, FCRKPM_OP_UH, p, b, 1, st);
                apply_one<double>(c, FCRKPM_OP_K_FULL, p, kp, 1, st);
                ++products;
                launch_lincomb_masked(kd, 1.0, fr, -1.0, nullptr, c.chi, t, nn, 1, st);
                dots<double>(c, t, p, 1, S_NORM, st);
                dots<double>(c, kp, p, 1, S_BB, st);
                const double* h = read_scalars(c, 1, st);
                c0 = h[S_NORM];
                c1 = h[S_BB];
            } else {
                apply_grad(c, p, b, st);
                dots<double>(c, fr, p, 1, S_NORM, st);
                c0 = -read_scalars(c, 1, st)[S_NORM];
            }
            // phi'(alpha) = c0 + c1 alpha + q0 + q1 alpha + q2 alpha^2 + q3 alpha^3,
            // the q_j from one pass over the nodes; its root by safeguarded Newton
            // steps on the host (phi is convex along p: phi' increases, and
            // phi'(0) < 0 along a descent direction)
            launch_ls_poly(cubic ? 0 : 1, dim, a, b, vol, c.chi, kappa, nn, lsb, st);
            launch_reduce_to(lsb, nn, 4, lsb + 4 * kRedBlocks, st);
            double q[4];
            HIPCHK(hipMemcpyAsync(hq.data(), lsb + 4 * kRedBlocks, sizeof(double) * 4 * kScal,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int j = 0; j < 4; ++j) q[j] = hq[j * kScal];
            auto d1f = [&](double x) { return c0 + c1 * x + q[0] + x * (q[1] + x * (q[2] + x * q[3])); };
            auto d2f = [&](double x) { return c1 + q[1] + x * (2.0 * q[2] + 3.0 * x * q[3]); };
            double alpha = 0.0, lo = 0.0, hi = HUGE_VAL;
            bool polish = false;  // one more step once the steps are at 1e-12 of alpha
            for (int k = 0; k < 60; ++k) {
                const double d1 = d1f(alpha), d2 = d2f(alpha);
                ++lsteps;
                if (!std::isfinite(d1) || !(d2 > 0.0) || d1 == 0.0) break;
                if (d1 < 0.0) lo = alpha;
                else hi = alpha;
                double next = alpha - d1 / d2;
                if (!(next > lo && next < hi)) next = std::isfinite(hi) ? 0.5 * (lo + hi) : 2.0 * lo + 1.0;
                const double step = next - alpha;
                alpha = next;
                if (polish) break;
                polish = fabs(step) <= 1e-12 * fabs(alpha);
            }
            if (!std::isfinite(alpha)) break;
            launch_lincomb_masked(d, 1.0, p, alpha, nullptr, c.chi, d, nn, 1, st);
            launch_lincomb_masked(a, 1.0, b, alpha, nullptr, c.chi, a, nn, cubic ? 1 : dim, st);
            if (cubic) launch_lincomb_masked(kd, 1.0, kp, alpha, nullptr, c.chi, kd, nn, 1, st);
            // the new residual, then the Polak-Ribiere direction
            HIPCHK(hipMemcpyAsync(ro, rr, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
            residual();
            dots<double>(c, rr, rr, 1, S_NORM, st);
            dots<double>(c, rr, ro, 1, S_BB, st);
            const double* h = read_scalars(c, 1, st);
            const double rn_new = h[S_NORM];
            const double beta = rn > 0.0 ? std::max(0.0, (rn_new - h[S_BB]) / rn) : 0.0;
            launch_lincomb_masked(rr, 1.0, p, beta, nullptr, c.freem, p, nn, 1, st);
            rn = rn_new;
            ++it;
            if (!std::isfinite(rn)) break;
        }
        conv = conv || sqrt(rn) <= tol * fnorm;
        HIPCHK(hipMemcpyAsync(d_inout, d, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
        if (uh_out) apply_one<double>(c, FCRKPM_OP_UH, d, uh_out, 1, st);
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (info) {
            memset(info, 0, sizeof(*info));
            info->iters = it;
            info->outer_iters = lsteps;
            info->rel_res = info->true_rel_res = fnorm > 0.0 ? sqrt(rn) / fnorm : 0.0;
            info->matvecs_f64 = products;
        }
        if (log_enabled())
            fprintf(stderr, "[fcrkpm] nonlinear CG (%s): %d iterations, %d line-search steps, |R|/|f| %.3e\n",
                    cubic ? "cubic" : "gradient", it, lsteps, fnorm > 0.0 ? sqrt(rn) / fnorm : 0.0);
        if (!conv) {
            c.err = "nonlinear CG did not reach tol within maxit iterations";
            return FCRKPM_ERR_NOCONV;
        }
        return FCRKPM_OK;
    });
}

// -lap u + kappa u^3 = r with d = g on the Dirichlet nodes (Eq 8 with the term
// of Eq B.1): Newton's method on R(d) = K d + f^N(d) - f^r over the free rows,
// each step one solve of (K + N^T diag(3 kappa V u^2) N) delta = -R with the
// solver of fcrkpm_solve.  The Jacobian is a K-type product: the rows b^a,
// then b^0 weighted per node by sqrt(3 kappa) |u^h|.
extern "C" fcrkpm_status fcrkpm_solve_nonlinear(fcrkpm_ctx* ctx, int32_t mode, double kappa,
                                                const double* r, const double* g,
                                                double* d_inout, double* uh_out, double tol,
                                                double newton_tol, int32_t maxnewton,
                                                int32_t maxit, fcrkpm_info* info, void* stream)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        check_solve_args(mode, 1, tol, maxit);
        if (!r || !d_inout) fail(FCRKPM_ERR_ARG, "NULL array");
        if (!(kappa >= 0.0) || !std::isfinite(kappa)) fail(FCRKPM_ERR_ARG, "kappa must be finite and >= 0");
        if (!(newton_tol > 0.0) || maxnewton < 1) fail(FCRKPM_ERR_ARG, "newton_tol must be > 0 and maxnewton >= 1");
        hipStream_t st = (hipStream_t)stream;
        const long nn = c.nn;
        ensure_rhs(c, 1);
        ensure_work(c, 1);
        HIPCHK(hipMemsetAsync(c.dflag + 2, 0, sizeof(int), st));
        launch_check_finite(r, nn, c.dflag + 2, st);
        if (g) launch_check_finite(g, nn, c.dflag + 2, st);
        launch_check_finite(d_inout, nn, c.dflag + 2, st);
        int hf = 0;
        HIPCHK(hipMemcpyAsync(&hf, c.dflag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hf) fail(FCRKPM_ERR_ARG, "non-finite value in r, g or d");

        struct Buf {
            double* p = nullptr;
            ~Buf() { dfree(p); }
        } bufs;
        bufs.p = dalloc<double>((size_t)5 * nn);
        double* fr = bufs.p;          // f^r
        double* xn = fr + nn;         // free part of the Newton iterate
        double* dG = xn + nn;         // d_Gamma
        double* kd = dG + nn;         // chi_Omega f^r for its norm, then f^N
        double* fnl = kd + nn;        // kappa u^3, then the Jacobian weights 3 kappa u^2
        double* u = vec64(c, V_T);
        apply_one<double>(c, FCRKPM_OP_FR, r, fr, 1, st);
        if (g) launch_masked_copy<double>(g, c.dirm, dG, nn, 1, st);
        else HIPCHK(hipMemsetAsync(dG, 0, sizeof(double) * nn, st));
        launch_masked_copy<double>(d_inout, c.freem, xn, nn, 1, st);
        launch_lincomb_masked(fr, 1.0, nullptr, 0.0, nullptr, c.freem, kd, nn, 1, st);
        dots<double>(c, kd, kd, 1, S_BB, st);
        const double fnorm = sqrt(read_scalars(c, 1, st)[S_BB]);
        const double scale = fnorm > 0.0 ? fnorm : 1.0;

        fcrkpm_info acc;
        memset(&acc, 0, sizeof(acc));
        fcrkpm_status inner = FCRKPM_OK;
        bool conv = false;
        double rel = 0.0;
        for (int step = 0;; ++step) {
            launch_select(c.freem, xn, dG, d_inout, nn, 1, st);  // d = chi_Omega x + d_Gamma
            apply_one<double>(c, FCRKPM_OP_UH, d_inout, u, 1, st);
            launch_pow_scaled(u, kappa, 3, fnl, nn, st);
            apply_one<double>(c, FCRKPM_OP_FR, fnl, kd, 1, st);                  // f^N
            apply_one<double>(c, FCRKPM_OP_K_FULL, d_inout, vec64(c, V_Q), 1, st);  // K d
            double* b = vec64(c, V_B);  // -R = f^r - K d - f^N on the free rows
            launch_lincomb_masked(vec64(c, V_Q), -1.0, kd, -1.0, fr, c.freem, b, nn, 1, st);
            dots<double>(c, b, b, 1, S_NORM, st);
            rel = sqrt(read_scalars(c, 1, st)[S_NORM]) / scale;
            acc.outer_iters = step;
            if (log_enabled()) fprintf(stderr, "[fcrkpm] newton %d: |R| / |f| = %.3e\n", step, rel);
            if (rel <= newton_tol) {
                conv = true;
                break;
            }
            if (step == maxnewton) break;
            launch_pow_scaled(u, 3.0 * kappa, 2, fnl, nn, st);  // weights 3 kappa u^2
            HIPCHK(hipStreamSynchronize(st));
            free_set(c.jac_set);
            c.jac_set = make_set(c, 1.0, 1.0, st, fnl);
            HIPCHK(hipMemsetAsync(vec64(c, V_X), 0, sizeof(double) * nn, st));
            fcrkpm_info inf;
            {
                SetScope use(c, c.jac_set);
                Solver S(c, 1, mode, tol, maxit);
                run_solvers({&S}, graphs_enabled(c), st);
                const fcrkpm_status w = S.finish(&inf, st);
                if (w != FCRKPM_OK) inner = w;
            }
            acc.iters += inf.iters;
            acc.fallback_used |= inf.fallback_used;
            acc.matvecs_f64 += inf.matvecs_f64 + 1;
            acc.matvecs_f32 += inf.matvecs_f32;
            launch_lincomb_masked(xn, 1.0, vec64(c, V_X), 1.0, nullptr, c.freem, xn, nn, 1, st);
        }
        acc.rel_res = rel;
        acc.true_rel_res = rel;
        if (uh_out) apply_one<double>(c, FCRKPM_OP_UH, d_inout, uh_out, 1, st);
        HIPCHK(hipStreamSynchronize(st));
        free_set(c.jac_set);
        HIPCHK(hipGetLastError());
        if (info) *info = acc;
        if (!conv) {
            c.err = inner != FCRKPM_OK ? "a Newton step's linear solve did not reach the tolerance"
                                       : "Newton's method did not reach newton_tol";
            return FCRKPM_ERR_NOCONV;
        }
        return FCRKPM_OK;
    });
}

extern "C" fcrkpm_status fcrkpm_get_option(fcrkpm_ctx* ctx, int32_t option, int64_t* value)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        if (!value) fail(FCRKPM_ERR_ARG, "NULL value");
        switch (option) {
            case FCRKPM_OPT_GRAPHS: *value = c.use_graphs ? 1 : 0; break;
            case FCRKPM_OPT_REGPATH: *value = (c.use_regpath && reg_path_ok(c)) ? 1 : 0; break;
            case FCRKPM_OPT_REGLAYOUT: *value = c.reg_layout + 2 * (c.reg_tpw - 1); break;
            case FCRKPM_OPT_TUNE_NS0: *value = (int64_t)(1e6 * c.tune_ms[0]); break;
            case FCRKPM_OPT_TUNE_NS1: *value = (int64_t)(1e6 * c.tune_ms[1]); break;
            case FCRKPM_OPT_TUNE_NS2: *value = (int64_t)(1e6 * c.tune_ms[2]); break;
            case FCRKPM_OPT_TUNE_NS3: *value = (int64_t)(1e6 * c.tune_ms[3]); break;
            case FCRKPM_OPT_LINECONST: *value = (c.use_sym && c.sym) ? 1 : 0; break;
            case FCRKPM_OPT_SEP_LINES32: *value = c.sep_wcap[0]; break;
            case FCRKPM_OPT_SEP_LINES64: *value = c.sep_wcap[1]; break;
            case FCRKPM_OPT_TUNE_CACHED: *value = c.tune_cached ? 1 : 0; break;
            case FCRKPM_OPT_KN_REGPATH: *value = (use_reg_path64(c) && reg_kn_ok(c, nullptr)) ? 1 : 0; break;
            default: fail(FCRKPM_ERR_ARG, "unknown option");
        }
        return FCRKPM_OK;
    });
}

extern "C" fcrkpm_status fcrkpm_set_option(fcrkpm_ctx* ctx, int32_t option, int64_t value)
{
    if (!ctx) return FCRKPM_ERR_ARG;
    Ctx& c = ctx->c;
    return run_guarded(c.err, [&]() -> fcrkpm_status {
        switch (option) {
            case FCRKPM_OPT_GRAPHS:
                if (value != 0 && value != 1) fail(FCRKPM_ERR_ARG, "FCRKPM_OPT_GRAPHS takes 0 or 1");
                c.use_graphs = value == 1;
                break;
            case FCRKPM_OPT_REGPATH:
                if (value != 0 && value != 1) fail(FCRKPM_ERR_ARG, "FCRKPM_OPT_REGPATH takes 0 or 1");
                c.use_regpath = value == 1;
                break;
            case FCRKPM_OPT_REGLAYOUT:
                if (!((reg_path_ok(c) || reg_gpq_ok(c)) ? reg_variant_ok(c, (int)value) : value == 0))
                    fail(FCRKPM_ERR_ARG, "FCRKPM_OPT_REGLAYOUT out of range for this box");
                set_reg_variant(c, (int)value);
                break;
            case FCRKPM_OPT_LINECONST:
                if (value != 0 && value != 1) fail(FCRKPM_ERR_ARG, "FCRKPM_OPT_LINECONST takes 0 or 1");
                c.use_sym = value == 1;
                break;
            case FCRKPM_OPT_SEP_LINES32:
            case FCRKPM_OPT_SEP_LINES64:
                if (value != 16 && value != 8 && value != 4)
                    fail(FCRKPM_ERR_ARG, "lines per workgroup of the LDS-tiled passes: 16, 8 or 4");
                c.sep_wcap[option == FCRKPM_OPT_SEP_LINES64 ? 1 : 0] = (int)value;
                break;
            default:
                fail(FCRKPM_ERR_ARG, "unknown option");
        }
        return FCRKPM_OK;
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
            case FCRKPM_COEF_LUMPED_MASS: {
                // M^l = chi o F^-1[sum_p F(chi o V o b^0_p) o F(conj H_p)] (Eq C.13,
                // Alg C.2): the load vector of r = 1
                ensure_rhs(c, 1);
                ensure_work(c, 1);
                double* one = vec64(c, V_T);
                launch_mask_to_double(c.chi, one, c.nn, st);
                apply_one<double>(c, FCRKPM_OP_FR, one, out, 1, st);
                break;
            }
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
