// C ABI of the ddwc library: context, workspace, the global Krylov solver with FP64
// defect correction, the Schur-complement pipeline and the determinant-ratio estimator.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ddwc.h"
#include "ddwc_internal.h"

using namespace ddwc;

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HC(call)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(DDWC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

#define CK(expr)                 \
    do {                         \
        int st_ = (expr);        \
        if (st_ != DDWC_OK) return st_; \
    } while (0)

// ------------------------------------------------------------------ profiler
namespace ddwc {
hipEvent_t Profiler::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
}
void Profiler::begin(hipStream_t s, int kclass, double b, Pair& p) {
    if (pending.size() >= 4096) harvest();
    p.a = get();
    p.b = get();
    p.kclass = kclass;
    p.bytes = b;
    (void)hipEventRecord(p.a, s);
}
void Profiler::end(hipStream_t s, Pair& p) {
    (void)hipEventRecord(p.b, s);
    pending.push_back(p);
}
void Profiler::harvest() {
    for (auto& p : pending) {
        (void)hipEventSynchronize(p.b);
        float ms_ = 0;
        if (hipEventElapsedTime(&ms_, p.a, p.b) == hipSuccess) {
            ms[p.kclass] += ms_;
            launches[p.kclass] += 1;
            bytes[p.kclass] += p.bytes;
        }
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
}
void Profiler::reset() {
    harvest();
    for (int k = 0; k < 8; ++k) {
        launches[k] = 0;
        ms[k] = 0;
        bytes[k] = 0;
    }
}
Profiler::~Profiler() {
    harvest();
    for (auto e : pool) (void)hipEventDestroy(e);
}
}  // namespace ddwc

// ------------------------------------------------------------------ static device scratch
// Scratch of ddwc_dslash_apply_noalloc, for callers that cannot allocate device memory: the
// internal-layout input and output fields of one call.  Each GPU the library runs on holds its
// own copy for the life of the process; host code never uses the array's name as a device
// address, only the per-device address that hipGetSymbolAddress returns (scratch_address).
static constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_addr;  // device -> its copy of `scratch`

// Address of `scratch` on `device`, which must be the current device (looked up once per device).
static int scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return DDWC_OK;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(DDWC_EHIP, std::string("address of the static device scratch: ") + hipGetErrorString(e));
    }
    g_scratch_addr[device] = p;
    *out = p;
    return DDWC_OK;
}

// ------------------------------------------------------------------ context
struct ddwc_ctx {
    Geom g;
    int lat[4], blk[4];
    int device = 0;
    double csw = 0;
    double links_fp = 0;  // fingerprint of the canonical links (equal links give equal values)
    cx<double>* U64 = nullptr;
    cx<float>* U32 = nullptr;
    cx<float>* U32s = nullptr;  // own-site FP32 link records [V][8][9] (RHS-innermost full Dslash)
    double2* K64 = nullptr;
    float4* K32 = nullptr;
    int* nbr = nullptr;  // neighbour table [8][V]
    // even-odd half fields (allocated when every block extent is even)
    cx<double>* Uh64 = nullptr;
    cx<float>* Uh32 = nullptr;
    double2* Kh64 = nullptr;
    cx<f16>* Uh16 = nullptr;  // FP16 half-order links (storage of the FP16 inner solver)
    cx<float>* Uh32s = nullptr;  // own-site link records [2][V/2][8][9] (FP32, FP16) read by the
    cx<f16>* Uh16s = nullptr;    // RHS-innermost kernels of the global solver
    float4* Kh32 = nullptr;
    int* nbr_eo = nullptr;
    struct Ainv {
        double mass4;
        double2* a64;
        float4* a32;
        unsigned long long used;
    };
    std::vector<Ainv> ainv;  // odd-site inverses of 4 + m + C for the masses in use
    unsigned long long clock = 0;
    Profiler prof;
    struct Buf {
        void* p = nullptr;
        size_t n = 0;
    };
    std::map<std::string, Buf> ws;
    double* host = nullptr;  // pinned scratch for small device-to-host copies
    void* blas = nullptr;    // dense linear-algebra handle (block determinants), created on first use
    // schedule options (ddwc_set_option, ddwc_autotune)
    int opt_graphs = 1;       // replay the global solver's iteration chunks from captured graphs
    int opt_poll = 2;         // BiCGStab iterations between host convergence checks
    int opt_inner_floor = 200;  // FP32 inner solves of the even-odd global solver stop at a relative
                                // residual of at least opt_inner_floor x 1e-8
    int opt_blk_threads = 0;  // block-solver workgroup size (0: default rule)
    int opt_solver = 0;       // global solver: 0 even-odd BiCGStab, 1 SAP-preconditioned GCR
    int opt_blk_lds = 0;      // KiB of LDS reserved per persistent block-solver workgroup
    int opt_blk_kernel = 0;   // block inner solver: 0 LDS-resident where it fits (FP32/FP16), 1 global-memory
    int opt_op_threads = WG;  // workgroup size of the global solver's RHS-innermost operator kernels
    int opt_tile_order = 1;   // their dispatch order: 0 half-site index order, 1 interleaved by block rank
    std::map<std::string, std::pair<int*, std::vector<int>>> orders;  // cached tile orders (device, host)
    int lds_max = 0;          // LDS bytes per workgroup of the device
    void* scratch = nullptr;  // this device's copy of the static scratch (ddwc_dslash_apply_noalloc)
    hipStream_t cap = nullptr;  // private stream the graphs are captured on
    struct Graph {
        std::vector<uintptr_t> key;
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        long long used = 0;
    };
    std::vector<Graph> graphs;
    size_t host_n = 0;
};

static int ws_get(ddwc_ctx* C, const std::string& key, size_t bytes, void** out) {
    auto& b = C->ws[key];
    if (b.n < bytes) {
        if (b.p) HC(hipFree(b.p));
        b.p = nullptr;
        b.n = 0;
        HC(hipMalloc(&b.p, bytes));
        b.n = bytes;
    }
    *out = b.p;
    return DDWC_OK;
}

template <class T>
static int ws_t(ddwc_ctx* C, const std::string& key, size_t count, T** out) {
    void* p;
    CK(ws_get(C, key, count * sizeof(T), &p));
    *out = (T*)p;
    return DDWC_OK;
}

static int host_buf(ddwc_ctx* C, size_t n, double** out) {
    if (C->host_n < n) {
        if (C->host) HC(hipHostFree(C->host));
        C->host = nullptr;
        HC(hipHostMalloc((void**)&C->host, n * sizeof(double)));
        C->host_n = n;
    }
    *out = C->host;
    return DDWC_OK;
}

static double mass_of(double kappa) { return 1.0 / (2.0 * kappa) - 4.0; }

static Exec make_exec(ddwc_ctx* C, void* stream) {
    Exec ex{(hipStream_t)stream, &C->prof, C->nbr};
    ex.blk_threads = C->opt_blk_threads;
    ex.blk_lds = C->opt_blk_lds;
    return ex;
}

static int check_ctx(const ddwc_ctx* C) {
    if (!C) return fail(DDWC_EINVAL, "null context");
    return DDWC_OK;
}

static int check_common(const ddwc_ctx* C, double kappa, int nrhs, int prec) {
    CK(check_ctx(C));
    if (!(kappa > 0) || !isfinite(kappa)) return fail(DDWC_EINVAL, "kappa must be positive and finite");
    if (nrhs < 1 || nrhs > 65535) return fail(DDWC_EINVAL, "nrhs must be in [1, 65535]");
    if (prec != DDWC_FP64 && prec != DDWC_MIXED32 && prec != DDWC_MIXED16) return fail(DDWC_EINVAL, "unknown precision");
    size_t words = (size_t)nrhs * 12 * C->g.V;
    if (words > (size_t)1 << 40) return fail(DDWC_EINVAL, "problem too large");
    return DDWC_OK;
}

// RHS-innermost fields address (site, RHS) element i * nrhs + r of a component plane with a
// 32-bit byte offset (at() in ddwc_device.h): usable while one plane of n * nrhs 16-byte words
// stays within 4 GiB.  Otherwise the fields are RHS-major.
static bool ri_fits(unsigned n, int nrhs) { return (uint64_t)n * (uint64_t)nrhs * 16u <= ((uint64_t)1 << 32); }

// The FP16 inner solver of the even-odd global solve needs RHS-innermost fields of at most WG RHS;
// checked at every entry point that can reach it, before any launch.
static int check_h16_global(const ddwc_ctx* C, int nrhs, int prec) {
    if (prec != DDWC_MIXED16 || !C->g.eo || C->opt_solver != 0) return DDWC_OK;
    if (nrhs > WG || !ri_fits((unsigned)(C->g.V / 2), nrhs))
        return fail(DDWC_EINVAL, "the FP16 inner solver takes at most 256 RHS (and V/2 * nrhs <= 2^28)");
    return DDWC_OK;
}

static size_t vec_words(const ddwc_ctx* C, int nrhs, bool fp64) {
    return (size_t)nrhs * (fp64 ? 12 : 6) * C->g.V;  // 16-byte words
}

double ddwc_dslash_bytes(const ddwc_ctx* C, int nrhs, int prec) {
    if (!C) return 0;
    const double r = prec == DDWC_FP64 ? 8.0 : 4.0;
    // per site: spinor in + out (24 reals each per RHS), 4 links (72 reals), clover (72 reals)
    return (double)C->g.V * ((double)nrhs * 48.0 * r + 144.0 * r);
}

extern "C" int ddwc_create(ddwc_ctx** out, const int lat[4], const int blk[4], int time_bc, double c_sw,
                           const void* links_dev, void* stream) {
    if (!out || !lat || !blk || !links_dev) return fail(DDWC_EINVAL, "null argument");
    *out = nullptr;
    if (time_bc != -1 && time_bc != 1) return fail(DDWC_EINVAL, "time_bc must be -1 or +1");
    if (!isfinite(c_sw)) return fail(DDWC_EINVAL, "c_sw must be finite");
    long long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (lat[mu] < 1 || blk[mu] < 1 || lat[mu] % blk[mu] != 0)
            return fail(DDWC_EINVAL, "block extent must divide the lattice extent in every direction");
        int nb = lat[mu] / blk[mu];
        if (nb < 2 || nb % 2 != 0)
            return fail(DDWC_EINVAL, "the number of blocks in every direction must be even and >= 2");
        V *= lat[mu];
    }
    if (V * 12 * 16 > ((long long)1 << 40) || V > (1 << 30)) return fail(DDWC_EINVAL, "lattice too large");
    ddwc_ctx* C = new ddwc_ctx();
    C->g = make_geom(lat, blk, time_bc);
    const Geom& g = C->g;
    for (int mu = 0; mu < 4; ++mu) {
        C->lat[mu] = lat[mu];
        C->blk[mu] = blk[mu];
    }
    C->csw = c_sw;
    hipError_t e0 = hipGetDevice(&C->device);
    if (e0 == hipSuccess) e0 = hipDeviceGetAttribute(&C->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, C->device);
    if (e0 == hipSuccess && scratch_address(C->device, &C->scratch) != DDWC_OK) {
        delete C;
        return DDWC_EHIP;
    }
    size_t n = (size_t)4 * 9 * g.V;
    if (e0 != hipSuccess || hipMalloc(&C->U64, n * sizeof(cx<double>)) != hipSuccess ||
        hipMalloc(&C->U32, n * sizeof(cx<float>)) != hipSuccess ||
        hipMalloc(&C->U32s, 2 * n * sizeof(cx<float>)) != hipSuccess ||
        hipMalloc(&C->K64, (size_t)36 * g.V * sizeof(double2)) != hipSuccess ||
        hipMalloc(&C->K32, (size_t)18 * g.V * sizeof(float4)) != hipSuccess ||
        hipMalloc(&C->nbr, (size_t)8 * g.V * sizeof(int)) != hipSuccess) {
        ddwc_destroy(C);
        return fail(DDWC_EHIP, "device allocation of links/clover failed");
    }
    Exec ex = make_exec(C, stream);
    launch_nbr_build(ex, g, C->nbr);
    launch_links_import(ex, g, links_dev, C->U64, C->U32);
    launch_links_own(ex, (unsigned)g.V, C->U32, C->U32, C->nbr, C->U32s);
    launch_clover_build(ex, g, C->U64, c_sw, C->K64, C->K32);
    if (g.eo) {
        const size_t n2 = g.V / 2;
        if (hipMalloc(&C->Uh64, (size_t)2 * 36 * n2 * sizeof(cx<double>)) != hipSuccess ||
            hipMalloc(&C->Uh32, (size_t)2 * 36 * n2 * sizeof(cx<float>)) != hipSuccess ||
            hipMalloc(&C->Kh64, (size_t)2 * 36 * n2 * sizeof(double2)) != hipSuccess ||
            hipMalloc(&C->Kh32, (size_t)2 * 18 * n2 * sizeof(float4)) != hipSuccess ||
            hipMalloc(&C->nbr_eo, (size_t)2 * 8 * n2 * sizeof(int)) != hipSuccess ||
            hipMalloc(&C->Uh16, (size_t)2 * 36 * n2 * sizeof(cx<f16>)) != hipSuccess ||
            hipMalloc(&C->Uh32s, (size_t)2 * 72 * n2 * sizeof(cx<float>)) != hipSuccess ||
            hipMalloc(&C->Uh16s, (size_t)2 * 72 * n2 * sizeof(cx<f16>)) != hipSuccess) {
            ddwc_destroy(C);
            return fail(DDWC_EHIP, "device allocation of the even-odd fields failed");
        }
        launch_eo_setup(ex, g, C->U64, C->K64, C->nbr, C->Uh64, C->Uh32, C->Kh64, C->Kh32, C->nbr_eo);
        launch_eo_links_own(ex, (unsigned)n2, C->Uh32, C->nbr_eo, C->Uh32s);
        launch_links_to_half(ex, (size_t)2 * 36 * n2, C->Uh32, C->Uh16);
        launch_links_to_half(ex, (size_t)2 * 72 * n2, C->Uh32s, C->Uh16s);
    }
    double* fpp = nullptr;
    if (ws_t(C, "fp_part", FP_BLOCKS, &fpp) != DDWC_OK) {
        ddwc_destroy(C);
        return fail(DDWC_EHIP, "device allocation failed");
    }
    launch_link_fp(ex, links_dev, n, fpp);
    std::vector<double> fph(FP_BLOCKS);
    hipError_t e1 = hipGetLastError();
    hipError_t e3 = hipMemcpyAsync(fph.data(), fpp, sizeof(double) * FP_BLOCKS, hipMemcpyDeviceToHost, ex.stream);
    hipError_t e2 = hipStreamSynchronize((hipStream_t)stream);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        ddwc_destroy(C);
        hipError_t eb = e1 != hipSuccess ? e1 : (e3 != hipSuccess ? e3 : e2);
        return fail(DDWC_EHIP, std::string("setup kernels failed: ") + hipGetErrorString(eb));
    }
    for (int k = 0; k < FP_BLOCKS; ++k) C->links_fp += fph[k];
    *out = C;
    return DDWC_OK;
}

extern "C" int ddwc_destroy(ddwc_ctx* C) {
    if (C && C->blas) blas_handle_destroy(C->blas);
    if (C) {
        for (auto& gr : C->graphs) {
            if (gr.x) (void)hipGraphExecDestroy(gr.x);
            if (gr.g) (void)hipGraphDestroy(gr.g);
        }
        if (C->cap) (void)hipStreamDestroy(C->cap);
    }
    if (!C) return DDWC_OK;
    (void)hipDeviceSynchronize();
    C->prof.harvest();
    if (C->U64) (void)hipFree(C->U64);
    if (C->U32) (void)hipFree(C->U32);
    if (C->U32s) (void)hipFree(C->U32s);
    if (C->K64) (void)hipFree(C->K64);
    if (C->K32) (void)hipFree(C->K32);
    if (C->nbr) (void)hipFree(C->nbr);
    for (void* q : {(void*)C->Uh64, (void*)C->Uh32, (void*)C->Kh64, (void*)C->Kh32, (void*)C->nbr_eo, (void*)C->Uh16,
                    (void*)C->Uh32s, (void*)C->Uh16s})
        if (q) (void)hipFree(q);
    for (auto& a : C->ainv) {
        (void)hipFree(a.a64);
        (void)hipFree(a.a32);
    }
    for (auto& kv : C->ws)
        if (kv.second.p) (void)hipFree(kv.second.p);
    for (auto& kv : C->orders) (void)hipFree(kv.second.first);
    if (C->host) (void)hipHostFree(C->host);
    delete C;
    return DDWC_OK;
}

// ------------------------------------------------------------------ global solver
// FP64 defect correction around BiCGStab in precision R on all RHS at once.
// b64, x64: internal FP64 multi-vectors.  Scalars stay on the device; the host polls
// the per-RHS state every `poll` iterations.
struct SolveInfo {
    int outer = 0, inner = 0;
    double relres = 0;
};

template <class R>
static int global_solve(ddwc_ctx* C, Exec& ex, double mass, const double2* b64, double2* x64, int nrhs, double tol,
                        int maxit, SolveInfo* info) {
    typedef typename Traits<R>::word W;
    const Geom& g = C->g;
    const bool fp64 = sizeof(R) == 8;
    const size_t nw = vec_words(C, nrhs, fp64);
    const int nt = tiles_of(g.V);
    const cx<R>* U = fp64 ? (const cx<R>*)C->U64 : (const cx<R>*)C->U32;
    const W* K = fp64 ? (const W*)C->K64 : (const W*)C->K32;
    const int kcl = fp64 ? DDWC_K_DSLASH64 : DDWC_K_DSLASH32;
    const double dbytes = ddwc_dslash_bytes(C, nrhs, fp64 ? DDWC_FP64 : DDWC_MIXED32);
    const double rb = (double)nrhs * g.V * 24.0 * sizeof(R);  // one vector of nrhs spinors
    const double mass4 = 4.0 + mass;
    W *r, *rh, *p, *v, *s, *t, *xR;
    double2* r64;
    double *part, *sums, *scale, *thr;
    BiState* st;
    const std::string pre = fp64 ? "g64_" : "g32_";
    CK(ws_t(C, pre + "r", nw, &r));
    CK(ws_t(C, pre + "rh", nw, &rh));
    CK(ws_t(C, pre + "p", nw, &p));
    CK(ws_t(C, pre + "v", nw, &v));
    CK(ws_t(C, pre + "s", nw, &s));
    CK(ws_t(C, pre + "t", nw, &t));
    CK(ws_t(C, pre + "x", nw, &xR));
    CK(ws_t(C, "g_r64", vec_words(C, nrhs, true), &r64));
    CK(ws_t(C, "g_part", (size_t)nt * nrhs * NPART, &part));
    CK(ws_t(C, "g_sums", (size_t)nrhs * NPART, &sums));
    CK(ws_t(C, "g_scale", (size_t)nrhs, &scale));
    CK(ws_t(C, "g_thr", (size_t)nrhs, &thr));
    CK(ws_t(C, "g_state", (size_t)nrhs, &st));
    double* hb;
    const size_t nst = (sizeof(BiState) + 7) / 8;
    CK(host_buf(C, (size_t)nrhs * (NPART + 2 + nst) + 16, &hb));
    double* h_sums = hb;
    double* h_scale = hb + (size_t)nrhs * NPART;
    double* h_thr = h_scale + nrhs;
    BiState* h_st = (BiState*)(h_thr + nrhs);
    hipStream_t sm = ex.stream;

    // ||b||^2
    launch_dots(ex, g, b64, b64, part, nrhs);
    launch_finalize(ex, part, nt, nrhs, sums, nullptr, ST_SUM, nullptr);
    HC(hipMemcpyAsync(h_sums, sums, sizeof(double) * nrhs * NPART, hipMemcpyDeviceToHost, sm));
    HC(hipStreamSynchronize(sm));
    std::vector<double> bb(nrhs), rr(nrhs);
    for (int k = 0; k < nrhs; ++k) {
        bb[k] = h_sums[k * NPART + 2];
        rr[k] = bb[k];
        if (!isfinite(bb[k])) return fail(DDWC_ENONFINITE, "non-finite right-hand side");
    }
    HC(hipMemsetAsync(x64, 0, sizeof(double2) * vec_words(C, nrhs, true), sm));
    HC(hipMemcpyAsync(r64, b64, sizeof(double2) * vec_words(C, nrhs, true), hipMemcpyDeviceToDevice, sm));
    const double floor_eps = fp64 ? 0.0 : 2e-6;
    const int poll = 2;
    int total = 0, nout = 0;
    bool converged = false;
    while (true) {
        bool all = true;
        for (int k = 0; k < nrhs; ++k)
            if (bb[k] > 0 && rr[k] > tol * tol * bb[k]) all = false;
        if (all) {
            converged = true;
            break;
        }
        if (total >= maxit || nout >= 100) break;
        ++nout;
        for (int k = 0; k < nrhs; ++k) {
            bool done = !(bb[k] > 0 && rr[k] > tol * tol * bb[k]);
            h_scale[k] = done ? 0.0 : 1.0 / sqrt(rr[k]);
            double eps = done ? 0.0 : 0.5 * tol * sqrt(bb[k] / rr[k]);
            if (eps < floor_eps) eps = floor_eps;
            h_thr[k] = done ? 2.0 : eps * eps;
        }
        HC(hipMemcpyAsync(scale, h_scale, sizeof(double) * nrhs, hipMemcpyHostToDevice, sm));
        HC(hipMemcpyAsync(thr, h_thr, sizeof(double) * nrhs, hipMemcpyHostToDevice, sm));
        launch_bicg_init<R>(ex, g.V, false, r64, scale, r, rh, p, xR, part, nrhs);
        launch_finalize(ex, part, nt, nrhs, nullptr, st, ST_INIT, thr);
        int it = 0;
        while (total < maxit) {
            for (int k = 0; k < poll && total < maxit; ++k, ++it, ++total) {
                launch_dslash_dot<R>(ex, g, U, K, mass4, p, v, rh, part, nrhs, kcl, dbytes + rb);
                launch_finalize(ex, part, nt, nrhs, nullptr, st, ST_ALPHA, nullptr);
                launch_bicg_s<R>(ex, g.V, false, st, r, v, s, nrhs);
                launch_dslash_dot4<R>(ex, g, U, K, mass4, s, t, rh, part, nrhs, kcl, dbytes + rb);
                launch_finalize(ex, part, nt, nrhs, nullptr, st, ST_OMEGA, nullptr);
                launch_bicg_xrp<R>(ex, g.V, false, st, xR, p, s, t, v, r, part, nrhs);
                launch_finalize(ex, part, nt, nrhs, nullptr, st, ST_RR, nullptr);
            }
            HC(hipGetLastError());
            HC(hipMemcpyAsync(h_st, st, sizeof(BiState) * nrhs, hipMemcpyDeviceToHost, sm));
            HC(hipStreamSynchronize(sm));
            bool any = false;
            for (int k = 0; k < nrhs; ++k) any = any || h_st[k].active;
            if (!any) break;
        }
        launch_accumulate<R>(ex, g.V, false, xR, scale, x64, nrhs);
        launch_residual<double>(ex, g, C->U64, C->K64, mass4, x64, b64, r64, part, nrhs, DDWC_K_DSLASH64,
                                ddwc_dslash_bytes(C, nrhs, DDWC_FP64) + (double)nrhs * g.V * 192.0);
        launch_finalize(ex, part, nt, nrhs, sums, nullptr, ST_SUM, nullptr, 1);
        HC(hipMemcpyAsync(h_sums, sums, sizeof(double) * nrhs * NPART, hipMemcpyDeviceToHost, sm));
        HC(hipStreamSynchronize(sm));
        for (int k = 0; k < nrhs; ++k) {
            rr[k] = h_sums[k * NPART];
            if (!isfinite(rr[k])) return fail(DDWC_ENONFINITE, "non-finite residual in the global solve");
        }
    }
    double worst = 0;
    for (int k = 0; k < nrhs; ++k)
        if (bb[k] > 0) worst = fmax(worst, sqrt(rr[k] / bb[k]));
    if (info) {
        info->outer += nout;
        info->inner += total;
        info->relres = fmax(info->relres, worst);
    }
    if (!converged) return fail(DDWC_ENOCONV, "global solve did not reach its tolerance within maxit");
    return DDWC_OK;
}

// ------------------------------------------------------------------ even-odd global solver
// Half-field operator data.  site_major selects the own-site link records (FP32, FP16) that the
// RHS-innermost kernels of the global solver read (U[p]: the records of parity p); the block
// solver and FP64 read entry-major links.
template <class R>
static EoFields<R> eo_fields(const ddwc_ctx* C, bool site_major = false);
template <>
EoFields<double> eo_fields<double>(const ddwc_ctx* C, bool) {
    EoFields<double> F;
    F.n2 = C->g.V / 2;
    F.op_threads = C->opt_op_threads;
    for (int p = 0; p < 2; ++p) {
        F.U[p] = C->Uh64 + (size_t)p * 36 * F.n2;
        F.K[p] = C->Kh64 + (size_t)p * 36 * F.n2;
        F.nbr[p] = C->nbr_eo + (size_t)p * 8 * F.n2;
    }
    return F;
}
template <>
EoFields<float> eo_fields<float>(const ddwc_ctx* C, bool site_major) {
    EoFields<float> F;
    F.n2 = C->g.V / 2;
    F.op_threads = C->opt_op_threads;
    for (int p = 0; p < 2; ++p) {
        F.U[p] = site_major ? C->Uh32s + (size_t)p * 72 * F.n2 : C->Uh32 + (size_t)p * 36 * F.n2;
        F.K[p] = C->Kh32 + (size_t)p * 18 * F.n2;
        F.nbr[p] = C->nbr_eo + (size_t)p * 8 * F.n2;
    }
    return F;
}

template <>
EoFields<H16> eo_fields<H16>(const ddwc_ctx* C, bool site_major) {
    EoFields<H16> F;
    F.n2 = C->g.V / 2;
    F.op_threads = C->opt_op_threads;
    for (int p = 0; p < 2; ++p) {
        F.U[p] = site_major ? C->Uh16s + (size_t)p * 72 * F.n2 : C->Uh16 + (size_t)p * 36 * F.n2;
        F.K[p] = C->Kh32 + (size_t)p * 18 * F.n2;
        F.nbr[p] = C->nbr_eo + (size_t)p * 8 * F.n2;
    }
    return F;
}

// Dispatch order of the tiles of the RHS-innermost operator kernels on fields of n2 sites with
// per_block sites per block (half or full fields; nrhs RHS, nt pairs per tile): sorted by the
// block rank of their first site, then by colour.
// Blocks of the two colours with the same rank are neighbours along x3 (block_base), and after
// the XCD remap each XCD takes a contiguous run of ranks (a time layer at 48x24^3), so a block's
// face neighbours of the other colour are processed on the same XCD at nearly the same time,
// while in index order they are on another XCD.
static int tile_order(ddwc_ctx* C, unsigned n2, int nrhs, int nt, const int** out, int per_block = 0) {
    const Geom& g = C->g;
    if (per_block == 0) per_block = g.hvb;  // half fields; full fields pass Vb
    const std::string key = std::to_string(n2) + "/" + std::to_string(nrhs) + "/" + std::to_string(nt) + "/" +
                            std::to_string(per_block);
    auto it = C->orders.find(key);
    if (it == C->orders.end()) {
        const long long pairs = (long long)n2 * nrhs;
        const int ntiles = (int)((pairs + nt - 1) / nt);
        std::vector<std::pair<long long, int>> keys(ntiles);
        for (int t = 0; t < ntiles; ++t) {
            const long long b = ((long long)t * nt / nrhs) / per_block;  // colour-major block of the first pair
            const long long c = b / g.NBc, rank = b % g.NBc;
            keys[t] = {(rank * 2 + c) * (long long)ntiles + t, t};
        }
        std::sort(keys.begin(), keys.end());
        std::vector<int> ord(ntiles);
        for (int t = 0; t < ntiles; ++t) ord[t] = keys[t].second;
        int* d = nullptr;
        HC(hipMalloc(&d, sizeof(int) * ntiles));
        HC(hipMemcpy(d, ord.data(), sizeof(int) * ntiles, hipMemcpyHostToDevice));
        it = C->orders.emplace(key, std::make_pair(d, std::move(ord))).first;
    }
    *out = it->second.first;
    return DDWC_OK;
}

// Odd-site inverses of 4 + m + C for mass4 = 4 + m (kept for the last few masses).
static int get_ainv(ddwc_ctx* C, Exec& ex, double mass4, const double2** a64, const float4** a32) {
    const size_t n2 = C->g.V / 2;
    for (auto& a : C->ainv)
        if (a.mass4 == mass4) {
            a.used = ++C->clock;
            *a64 = a.a64;
            *a32 = a.a32;
            return DDWC_OK;
        }
    ddwc_ctx::Ainv* slot = nullptr;
    if (C->ainv.size() < 4) {
        ddwc_ctx::Ainv a{};
        HC(hipMalloc(&a.a64, (size_t)36 * n2 * sizeof(double2)));
        HC(hipMalloc(&a.a32, (size_t)18 * n2 * sizeof(float4)));
        C->ainv.push_back(a);
        slot = &C->ainv.back();
    } else {
        slot = &C->ainv[0];
        for (auto& a : C->ainv)
            if (a.used < slot->used) slot = &a;
    }
    slot->mass4 = mass4;
    slot->used = ++C->clock;
    launch_eo_inverse(ex, (unsigned)n2, C->Kh64 + (size_t)36 * n2, mass4, slot->a64, slot->a32);
    HC(hipGetLastError());
    *a64 = slot->a64;
    *a32 = slot->a32;
    return DDWC_OK;
}

// D(m) x = b with even-odd preconditioning: BiCGStab in precision R on
// Mee = A_ee - 1/4 H_eo A_oo^-1 H_oe inside FP64 defect correction, then
// x_o = A_oo^-1 (b_o + 1/2 H_oe x_e).  The FP64 residual of the even system equals the
// residual of the full system, so the stopping rule is ||b'_e - Mee x_e|| <= tol ||b||.
// The instantiated graph of the launches `body` issues, cached under `key` (at most 8 kept);
// captured on the context's private stream.  nullptr if capture is not possible.
template <class F>
static hipGraphExec_t graph_for(ddwc_ctx* C, const std::vector<uintptr_t>& key, F&& body) {
    static long long clock = 0;
    for (auto& gr : C->graphs)
        if (gr.key == key) {
            gr.used = ++clock;
            return gr.x;
        }
    if (!C->cap && hipStreamCreateWithFlags(&C->cap, hipStreamNonBlocking) != hipSuccess) {
        C->cap = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    Exec ec = make_exec(C, C->cap);
    ec.prof = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    if (hipStreamBeginCapture(C->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    body(ec);
    if (hipStreamEndCapture(C->cap, &g) != hipSuccess || !g ||
        hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return nullptr;
    }
    if (C->graphs.size() >= 8) {
        auto old = std::min_element(C->graphs.begin(), C->graphs.end(),
                                    [](const ddwc_ctx::Graph& a, const ddwc_ctx::Graph& b) { return a.used < b.used; });
        (void)hipGraphExecDestroy(old->x);
        (void)hipGraphDestroy(old->g);
        C->graphs.erase(old);
    }
    ddwc_ctx::Graph gr;
    gr.key = key;
    gr.g = g;
    gr.x = x;
    gr.used = ++clock;
    C->graphs.push_back(gr);
    return x;
}

template <class S>
static int eo_solve(ddwc_ctx* C, Exec& ex, double mass, const double2* b64, double2* x64, int nrhs, double tol,
                    int maxit, SolveInfo* info) {
    typedef typename Traits<S>::word W;
    typedef typename Traits<S>::real R;
    typedef typename Traits<S>::xs XS;
    typedef typename Traits<XS>::word XW;
    typedef typename Traits<S>::kword KW;
    const Geom& g = C->g;
    const bool fp64 = std::is_same<S, double>::value, h16 = std::is_same<S, H16>::value;
    const EoFields<double> F64 = eo_fields<double>(C);
    const unsigned n2 = F64.n2;
    Geom gh = g;  // geometry of the half fields for the vector kernels (only V is used)
    gh.V = (int)n2;
    const int nt = tiles_of(n2);
    const int ntf = tiles_of(g.V);
    // low-precision fields RHS-innermost: the RHS of a site share its links, clover and table
    // (FP16 fields, whose scale plane follows the word planes, always are)
    CK(check_h16_global(C, nrhs, h16 ? DDWC_MIXED16 : DDWC_MIXED32));
    const bool ri = h16 || (nrhs > 1 && nrhs <= WG && ri_fits(n2, nrhs));
    EoFields<S> FR = eo_fields<S>(C, ri && !fp64);  // RI kernels read own-site link records
    if (ri && g.eo && C->opt_tile_order == 1) CK(tile_order(C, n2, nrhs, eo_op_threads(FR, nrhs, ri), &FR.order));
    const int ntR = vector_tiles(n2, nrhs, ri);
    const int ntM = eo_op_tiles(FR, nrhs, ri);  // tiles of the operator kernels' partial sums
    const double mass4 = 4.0 + mass;
    const double2* A64;
    const float4* A32;
    CK(get_ainv(C, ex, mass4, &A64, &A32));
    const KW* AR = fp64 ? (const KW*)A64 : (const KW*)A32;
    const size_t hw64 = (size_t)nrhs * 12 * n2, stride = (size_t)nrhs * n2;
    // bytes of one precision-S field (FP16: three word planes and a plane of float scales)
    const size_t bytesR = h16 ? ((3 * 16 + 4) * stride + 15) / 16 * 16 : (size_t)Traits<S>::NCW * 16 * stride;
    const size_t bytesX = (size_t)Traits<XS>::NCW * 16 * stride;
    const int kcl = fp64 ? DDWC_K_DSLASH64 : DDWC_K_DSLASH32;
    // algorithmic bytes of one half operator (hop kernel): half input with neighbours, half
    // output, the links of all sites, the site matrix of one parity
    const double rs = h16 ? 52.0 : 24.0 * sizeof(R);
    const double hbytes =
        (double)n2 * (nrhs * 2 * rs + 8 * 18.0 * sizeof(typename Traits<S>::link) + 72.0 * sizeof(R));
    double2 *be, *bo, *bpe, *xe, *xo, *re, *to;
    W *r, *rh, *p, *v, *s, *t, *tmp;
    XW* xR;
    double *part, *sums, *scale, *thr;
    BiState* st;
    CK(ws_t(C, "eo_be", hw64, &be));
    CK(ws_t(C, "eo_bo", hw64, &bo));
    CK(ws_t(C, "eo_bpe", hw64, &bpe));
    CK(ws_t(C, "eo_xe", hw64, &xe));
    CK(ws_t(C, "eo_xo", hw64, &xo));
    CK(ws_t(C, "eo_re", hw64, &re));
    CK(ws_t(C, "eo_to", hw64, &to));
    const std::string pre = fp64 ? "eo64_" : h16 ? "eo16_" : "eo32_";
    {
        void* q;
        W** vecs[7] = {&r, &rh, &p, &v, &s, &t, &tmp};
        const char* nm[7] = {"r", "rh", "p", "v", "s", "t", "tmp"};
        for (int k = 0; k < 7; ++k) {
            CK(ws_get(C, pre + nm[k], bytesR, &q));
            *vecs[k] = (W*)q;
        }
        CK(ws_get(C, pre + "x", bytesX, &q));
        xR = (XW*)q;
    }
    CK(ws_t(C, "g_part", (size_t)std::max(ntf, std::max(ntR, ntM)) * nrhs * NPART, &part));
    CK(ws_t(C, "g_sums", (size_t)nrhs * NPART, &sums));
    CK(ws_t(C, "g_scale", (size_t)nrhs, &scale));
    CK(ws_t(C, "g_thr", (size_t)nrhs, &thr));
    CK(ws_t(C, "g_state", (size_t)nrhs, &st));
    double* hb;
    const size_t nst = (sizeof(BiState) + 7) / 8;
    CK(host_buf(C, (size_t)nrhs * (NPART + 2 + nst) + 16, &hb));
    double* h_sums = hb;
    double* h_scale = hb + (size_t)nrhs * NPART;
    double* h_thr = h_scale + nrhs;
    BiState* h_st = (BiState*)(h_thr + nrhs);
    hipStream_t sm = ex.stream;

    // ||b||^2 of the full system
    launch_dots(ex, g, b64, b64, part, nrhs);
    launch_finalize(ex, part, ntf, nrhs, sums, nullptr, ST_SUM, nullptr);
    HC(hipMemcpyAsync(h_sums, sums, sizeof(double) * nrhs * NPART, hipMemcpyDeviceToHost, sm));
    HC(hipStreamSynchronize(sm));
    std::vector<double> bb(nrhs), rr(nrhs);
    for (int k = 0; k < nrhs; ++k) {
        bb[k] = h_sums[k * NPART + 2];
        if (!isfinite(bb[k])) return fail(DDWC_ENONFINITE, "non-finite right-hand side");
    }
    // b'_e = b_e + 1/2 H_eo A_oo^-1 b_o ; x_e = 0 ; r_e = b'_e
    launch_eo_split(ex, g, b64, be, bo, nrhs);
    // t0 = A_oo^-1 b_o is kept: with the last residual's A_oo^-1 H x_e it gives x_o at the end
    launch_eo_hopinv<double>(ex, F64, 1, false, nullptr, bo, 0.0, A64, xo, nrhs, DDWC_K_OTHER, 0);
    launch_eo_diaghop<double>(ex, F64, 0, false, 0, false, be, xo, 0.5, 0.0, nullptr, bpe, nullptr, nrhs, DDWC_K_OTHER, 0);
    HC(hipMemsetAsync(xe, 0, sizeof(double2) * hw64, sm));
    HC(hipMemcpyAsync(re, bpe, sizeof(double2) * hw64, hipMemcpyDeviceToDevice, sm));
    launch_dots(ex, gh, re, re, part, nrhs);
    launch_finalize(ex, part, nt, nrhs, sums, nullptr, ST_SUM, nullptr);
    HC(hipMemcpyAsync(h_sums, sums, sizeof(double) * nrhs * NPART, hipMemcpyDeviceToHost, sm));
    HC(hipStreamSynchronize(sm));
    for (int k = 0; k < nrhs; ++k) rr[k] = h_sums[k * NPART + 2];
    // the inner solve stops at this relative residual at the least (the storage's reach)
    const double floor_eps = fp64 ? 0.0 : h16 ? 1e-3 : 1e-8 * C->opt_inner_floor;
    const int poll = C->opt_poll;
    int total = 0, nout = 0;
    bool converged = false;
    // `iters` BiCGStab iterations on stream ee (the caller's, or the capture stream)
    auto chunk = [&](Exec& ee, int iters) {
        auto apply_M = [&](const W* in, W* out, int epi, const W* aux) {
            launch_eo_hopinv<S>(ee, FR, 1, ri, in, nullptr, 1.0, AR, tmp, nrhs, fp64 ? kcl : DDWC_K_EOHOP, hbytes);
            launch_eo_diaghop<S>(ee, FR, 0, ri, epi, true, in, tmp, -0.25, mass4, aux, out, part, nrhs, kcl,
                                 hbytes + (double)nrhs * n2 * rs);
        };
        // BiCGStab (van der Vorst) with the next rho taken from the dot products of t = M s, so
        // that x, r and p are updated in one pass
        for (int k = 0; k < iters; ++k) {
            apply_M(p, v, 1, rh);
            launch_finalize(ee, part, ntM, nrhs, nullptr, st, ST_ALPHA, nullptr);
            launch_bicg_s<S>(ee, n2, ri, st, r, v, s, nrhs);
            apply_M(s, t, 2, rh);
            launch_finalize(ee, part, ntM, nrhs, nullptr, st, ST_OMEGA, nullptr);
            launch_bicg_xrp<S>(ee, n2, ri, st, xR, p, s, t, v, r, part, nrhs);
            launch_finalize(ee, part, ntR, nrhs, nullptr, st, ST_RR, nullptr);
        }
    };
    // a chunk of `poll` iterations replayed from a graph (every argument of its launches is in
    // the key, so one graph serves every chunk of every solve with the same buffers and mass)
    hipGraphExec_t gx = nullptr;
    if (C->opt_graphs && !C->prof.on) {
        double m4 = mass4;
        uint64_t mb;
        memcpy(&mb, &m4, 8);
        std::vector<uintptr_t> key = {(uintptr_t)(fp64 ? 1 : h16 ? 3 : 2), (uintptr_t)nrhs, (uintptr_t)ri,
                                      (uintptr_t)n2, (uintptr_t)poll, (uintptr_t)mb, (uintptr_t)r, (uintptr_t)rh,
                                      (uintptr_t)p, (uintptr_t)v, (uintptr_t)s, (uintptr_t)t, (uintptr_t)tmp,
                                      (uintptr_t)xR, (uintptr_t)part, (uintptr_t)st, (uintptr_t)AR,
                                      (uintptr_t)FR.U[0], (uintptr_t)FR.K[0], (uintptr_t)FR.op_threads,
                                      (uintptr_t)FR.order};
        gx = graph_for(C, key, [&](Exec& ee) { chunk(ee, poll); });
    }
    while (true) {
        bool all = true;
        for (int k = 0; k < nrhs; ++k)
            if (bb[k] > 0 && rr[k] > tol * tol * bb[k]) all = false;
        if (all) {
            converged = true;
            break;
        }
        if (total >= maxit || nout >= 100) break;
        ++nout;
        for (int k = 0; k < nrhs; ++k) {
            bool done = !(bb[k] > 0 && rr[k] > tol * tol * bb[k]);
            h_scale[k] = done ? 0.0 : 1.0 / sqrt(rr[k]);
            double eps = done ? 0.0 : 0.5 * tol * sqrt(bb[k] / rr[k]);
            if (eps < floor_eps) eps = floor_eps;
            h_thr[k] = done ? 2.0 : eps * eps;
        }
        HC(hipMemcpyAsync(scale, h_scale, sizeof(double) * nrhs, hipMemcpyHostToDevice, sm));
        HC(hipMemcpyAsync(thr, h_thr, sizeof(double) * nrhs, hipMemcpyHostToDevice, sm));
        launch_bicg_init<S>(ex, n2, ri, re, scale, r, rh, p, xR, part, nrhs);
        launch_finalize(ex, part, ntR, nrhs, nullptr, st, ST_INIT, thr);
        while (total < maxit) {
            const int it = std::min(poll, maxit - total);
            if (gx && it == poll)
                HC(hipGraphLaunch(gx, sm));
            else
                chunk(ex, it);
            total += it;
            HC(hipGetLastError());
            HC(hipMemcpyAsync(h_st, st, sizeof(BiState) * nrhs, hipMemcpyDeviceToHost, sm));
            HC(hipStreamSynchronize(sm));
            bool any = false;
            for (int k = 0; k < nrhs; ++k) any = any || h_st[k].active;
            if (!any) break;
        }
        launch_accumulate<S>(ex, n2, ri, xR, scale, xe, nrhs);
        // r_e = b'_e - Mee x_e in FP64
        launch_eo_hopinv<double>(ex, F64, 1, false, xe, nullptr, 1.0, A64, to, nrhs, DDWC_K_DSLASH64, 0);
        launch_eo_diaghop<double>(ex, F64, 0, false, 3, true, xe, to, -0.25, mass4, bpe, re, part, nrhs, DDWC_K_DSLASH64, 0);
        launch_finalize(ex, part, nt, nrhs, sums, nullptr, ST_SUM, nullptr, 1);
        HC(hipMemcpyAsync(h_sums, sums, sizeof(double) * nrhs * NPART, hipMemcpyDeviceToHost, sm));
        HC(hipStreamSynchronize(sm));
        for (int k = 0; k < nrhs; ++k) {
            rr[k] = h_sums[k * NPART];
            if (!isfinite(rr[k])) return fail(DDWC_ENONFINITE, "non-finite residual in the global solve");
        }
    }
    // x_o = A_oo^-1 (b_o + 1/2 H_oe x_e) = t0 + 1/2 (A_oo^-1 H_oe x_e), the second term from the
    // last residual pass (x_e = 0 when no outer step ran), x = (x_e, x_o)
    launch_eo_merge(ex, g, xe, xo, x64, nrhs, nout > 0 ? to : nullptr, 0.5);
    HC(hipGetLastError());
    double worst = 0;
    for (int k = 0; k < nrhs; ++k)
        if (bb[k] > 0) worst = fmax(worst, sqrt(rr[k] / bb[k]));
    if (info) {
        info->outer += nout;
        info->inner += total;
        info->relres = fmax(info->relres, worst);
    }
    if (!converged) return fail(DDWC_ENOCONV, "global solve did not reach its tolerance within maxit");
    return DDWC_OK;
}

static int sap_gcr(ddwc_ctx* C, Exec& ex, double mass, const double2* b64, double2* x64, int nrhs, double tol,
                   int maxit, int prec, SolveInfo* info);

static int solve_internal(ddwc_ctx* C, Exec& ex, double mass, const double2* b64, double2* x64, int nrhs,
                          double tol, int maxit, int prec, SolveInfo* info) {
    if (C->opt_solver == 1) return sap_gcr(C, ex, mass, b64, x64, nrhs, tol, maxit, prec, info);
    if (C->g.eo) {
        if (prec == DDWC_FP64) return eo_solve<double>(C, ex, mass, b64, x64, nrhs, tol, maxit, info);
        if (prec == DDWC_MIXED16) return eo_solve<H16>(C, ex, mass, b64, x64, nrhs, tol, maxit, info);
        return eo_solve<float>(C, ex, mass, b64, x64, nrhs, tol, maxit, info);
    }
    if (prec == DDWC_FP64) return global_solve<double>(C, ex, mass, b64, x64, nrhs, tol, maxit, info);
    return global_solve<float>(C, ex, mass, b64, x64, nrhs, tol, maxit, info);
}

// ------------------------------------------------------------------ block solves
struct BlockInfo {
    int outer = 0, inner = 0;
    double relres = 0;
    long long block_iters = 0;  // summed over blocks and RHS
};

// Floating-point operations of one inner BiCGStab iteration of a block solve, per even site (eo)
// or per block site: two applications of the block operator, each a pass over both parities
// (eo) or one full pass, with 180 flops per hop term (spin projection, two 3x3 complex
// products, reconstruction) over the hops that stay inside the block (2 sum_mu (b_mu - 1)/b_mu
// per site on average) and 540 per site for the two packed Hermitian 6x6 blocks, plus about 400
// for the vector updates and dot products.  The block class of the profiler accumulates this
// model: the block kernels work from LDS and the caches, so their roofline is the ALU.
static double block_flops_per_site(const Geom& g, bool eo) {
    double hops = 0;
    for (int mu = 0; mu < 4; ++mu) hops += 2.0 * (g.b[mu] - 1) / g.b[mu];
    const double pass = hops * 180.0 + 540.0;
    return 2.0 * (eo ? 2.0 : 1.0) * pass + 400.0;
}

// Even-odd preconditioned block solves (every block extent even): FP64 prep, then FP64
// defect-correction steps around the persistent inner solver until every block of the
// colour has ||b'_e - M_k x_e|| <= tol ||b_k||, then the odd sites.
static int block_internal_eo(ddwc_ctx* C, Exec& ex, int colour, double mass, const double2* b64, double2* x64,
                             int nrhs, double tol, int maxit, int prec, BlockInfo* info) {
    const Geom& g = C->g;
    const bool fp64 = prec == DDWC_FP64;
    const double mass4 = 4.0 + mass;
    const double2* A64;
    const float4* A32;
    CK(get_ainv(C, ex, mass4, &A64, &A32));
    const EoFields<double> F64 = eo_fields<double>(C);
    const unsigned n2 = F64.n2;
    // blocks whose parity fits the LDS-resident kernel run it in FP32 for both low precisions
    const bool lds = !fp64 && C->opt_blk_kernel == 0 && blk_lds_fits(g, C->lds_max);
    const bool h16 = prec == DDWC_MIXED16 && !lds;
    const size_t hw64 = (size_t)nrhs * 12 * n2;
    // the correction vector (slot 5) is kept in FP32 when the others are FP16
    const int sprec = lds ? DDWC_MIXED32 : prec;
    const size_t slabS = blk_slab_bytes(sprec, n2), slabX = blk_slab_bytes(h16 ? DDWC_MIXED32 : sprec, n2);
    double2 *bpe, *re, *xe, *to, *th;
    CK(ws_t(C, "be_bpe", hw64, &bpe));
    CK(ws_t(C, "be_re", hw64, &re));
    CK(ws_t(C, "be_xe", hw64, &xe));
    CK(ws_t(C, "be_to", hw64, &to));  // A_oo^-1 b_o (prep)
    CK(ws_t(C, "be_th", hw64, &th));  // A_oo^-1 H x_e of the last residual pass
    void* w[7];
    const char* names[7] = {"be_r", "be_rh", "be_p", "be_v", "be_t", "be_e", "be_tmp"};
    for (int k = 0; k < 7; ++k)
        CK(ws_get(C, std::string(names[k]) + (fp64 ? "64" : h16 ? "16" : "32"), (k == 5 ? slabX : slabS) * nrhs,
                  &w[k]));
    // (the LDS-resident kernel uses slots 1, 3, 5 only)
    const size_t nb = (size_t)nrhs * g.NBc;
    double *bb, *rr;
    int* iters;
    CK(ws_t(C, "be_bb", nb, &bb));
    CK(ws_t(C, "be_rr", nb, &rr));
    CK(ws_t(C, "be_iters", nb, &iters));
    HC(hipMemsetAsync(iters, 0, nb * sizeof(int), ex.stream));
    // (k_blk_recon writes this colour's solution and clears the other colour)
    launch_blk_prep(ex, g, F64, A64, b64, bpe, re, xe, to, bb, rr, colour, nrhs);
    std::vector<double> hbb(nb), hrr(nb);
    std::vector<int> hit(nb);
    HC(hipMemcpyAsync(hbb.data(), bb, nb * sizeof(double), hipMemcpyDeviceToHost, ex.stream));
    int nout = 0, imax = 0;
    long long isum = 0;
    bool converged = false, finite = true;
    while (true) {
        HC(hipMemcpyAsync(hrr.data(), rr, nb * sizeof(double), hipMemcpyDeviceToHost, ex.stream));
        HC(hipMemcpyAsync(hit.data(), iters, nb * sizeof(int), hipMemcpyDeviceToHost, ex.stream));
        HC(hipStreamSynchronize(ex.stream));
        bool all = true;
        imax = 0;
        isum = 0;
        for (size_t k = 0; k < nb; ++k) {
            if (!isfinite(hrr[k]) || !isfinite(hbb[k])) finite = false;
            if (hbb[k] > 0 && hrr[k] > tol * tol * hbb[k]) all = false;
            imax = hit[k] > imax ? hit[k] : imax;
            isum += hit[k];
        }
        if (!finite) break;
        if (all) {
            converged = true;
            break;
        }
        if (imax >= maxit || nout >= 30) break;
        ++nout;
        if (fp64) {
            const EoFields<double> F = F64;
            launch_blk_inner<double>(ex, g, F, A64, re, xe, w, bb, rr, mass4, tol, maxit - imax, iters, colour, nrhs);
        } else if (lds) {
            const EoFields<float> F = eo_fields<float>(C);
            launch_blk_lds(ex, g, F, A32, re, xe, w, bb, rr, mass4, tol, maxit - imax, iters, colour, nrhs);
        } else if (h16) {
            const EoFields<H16> F = eo_fields<H16>(C);
            launch_blk_inner<H16>(ex, g, F, A32, re, xe, w, bb, rr, mass4, tol, maxit - imax, iters, colour, nrhs);
        } else {
            const EoFields<float> F = eo_fields<float>(C);
            launch_blk_inner<float>(ex, g, F, A32, re, xe, w, bb, rr, mass4, tol, maxit - imax, iters, colour, nrhs);
        }
        launch_blk_resid(ex, g, F64, A64, bpe, xe, re, th, rr, mass4, colour, nrhs);
    }
    // x_o = A_oo^-1 b_o + 1/2 A_oo^-1 H x_e from the prep and the last residual pass (x_e = 0 when
    // no inner solve ran)
    launch_blk_recon(ex, g, to, nout > 0 ? th : nullptr, xe, x64, colour, nrhs);
    HC(hipGetLastError());
    double worst = 0;
    for (size_t k = 0; k < nb; ++k)
        if (hbb[k] > 0) worst = fmax(worst, sqrt(hrr[k] / hbb[k]));
    if (info) {
        info->outer += nout;
        info->inner += imax;
        info->relres = fmax(info->relres, worst);
        info->block_iters += isum;
    }
    if (C->prof.on) C->prof.bytes[DDWC_K_BLOCK] += (double)isum * g.hvb * block_flops_per_site(g, true);
    if (!finite) return fail(DDWC_ENONFINITE, "non-finite residual in a block solve");
    if (!converged) return fail(DDWC_ENOCONV, "a block solve did not reach its tolerance within maxit");
    return DDWC_OK;
}

static int block_internal(ddwc_ctx* C, Exec& ex, int colour, double mass, const double2* b64, double2* x64,
                          int nrhs, double tol, int maxit, int prec, BlockInfo* info) {
    if (C->g.eo) return block_internal_eo(C, ex, colour, mass, b64, x64, nrhs, tol, maxit, prec, info);
    const Geom& g = C->g;
    const bool fp64 = prec == DDWC_FP64;
    const size_t nw = vec_words(C, nrhs, fp64);
    const size_t esz = 16;
    BlockSolveArgs a;
    a.b = b64;
    a.x = x64;
    CK(ws_t(C, "b_r64", vec_words(C, nrhs, true), &a.r64));
    const char* names[6] = {"b_r", "b_rh", "b_p", "b_v", "b_t", "b_e"};
    for (int k = 0; k < 6; ++k) CK(ws_get(C, std::string(names[k]) + (fp64 ? "64" : "32"), nw * esz, &a.w[k]));
    a.colour = colour;
    a.nrhs = nrhs;
    a.mass4 = 4.0 + mass;
    a.tol = tol;
    a.maxit = maxit;
    const size_t nb = (size_t)nrhs * g.NBc;
    CK(ws_t(C, "b_iters", nb, &a.iters));
    CK(ws_t(C, "b_outer", nb, &a.outer));
    CK(ws_t(C, "b_relres", nb, &a.relres));
    // the other colour of x is zero
    const size_t half = (size_t)g.V / 2;
    for (int k = 0; k < nrhs; ++k)
        for (int c = 0; c < 12; ++c)
            HC(hipMemsetAsync(x64 + ((size_t)k * 12 + c) * g.V + (colour == 0 ? half : 0), 0, half * sizeof(double2),
                              ex.stream));
    if (fp64)
        launch_block_solve64(ex, g, C->U64, C->K64, a);
    else
        launch_block_solve32(ex, g, C->U64, C->K64, C->U32, C->K32, a);
    HC(hipGetLastError());
    std::vector<int> it(nb), ou(nb);
    std::vector<double> rr(nb);
    HC(hipMemcpyAsync(it.data(), a.iters, nb * sizeof(int), hipMemcpyDeviceToHost, ex.stream));
    HC(hipMemcpyAsync(ou.data(), a.outer, nb * sizeof(int), hipMemcpyDeviceToHost, ex.stream));
    HC(hipMemcpyAsync(rr.data(), a.relres, nb * sizeof(double), hipMemcpyDeviceToHost, ex.stream));
    HC(hipStreamSynchronize(ex.stream));
    int imax = 0, omax = 0;
    double worst = 0;
    long long sum = 0;
    bool finite = true;
    for (size_t k = 0; k < nb; ++k) {
        imax = it[k] > imax ? it[k] : imax;
        omax = ou[k] > omax ? ou[k] : omax;
        if (!isfinite(rr[k])) finite = false;
        worst = fmax(worst, rr[k]);
        sum += it[k];
    }
    if (info) {
        info->outer += omax;
        info->inner += imax;
        info->relres = fmax(info->relres, worst);
        info->block_iters += sum;
    }
    if (C->prof.on) C->prof.bytes[DDWC_K_BLOCK] += (double)sum * g.Vb * block_flops_per_site(g, false);
    if (!finite) return fail(DDWC_ENONFINITE, "non-finite residual in a block solve");
    if (worst > tol) return fail(DDWC_ENOCONV, "a block solve did not reach its tolerance within maxit");
    return DDWC_OK;
}

// ------------------------------------------------------------------ public entry points
static void fill_stats(ddwc_stats* s, int outer, int inner, double rel, std::chrono::steady_clock::time_point t0) {
    if (!s) return;
    s->outer_iters = outer;
    s->inner_iters = inner;
    s->rel_residual = rel;
    s->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// out = D(m) in through internal-layout fields a and b (each dslash_field_bytes long): from the
// context's workspace, or from the static scratch for the no-allocation entry point.
static size_t dslash_field_bytes(const ddwc_ctx* C, int nrhs, int prec) {
    return vec_words(C, nrhs, prec == DDWC_FP64) * 16;
}
static int dslash_apply_with(ddwc_ctx* C, Exec& ex, double kappa, const void* in, void* out, int nrhs, int prec,
                             void* a, void* b, bool may_allocate) {
    const Geom& g = C->g;
    const double mass4 = 4.0 + mass_of(kappa);
    if (prec == DDWC_FP64) {
        launch_import<double>(ex, g, in, (double2*)a, nrhs, MASK_ALL);
        launch_dslash<double>(ex, g, C->U64, C->K64, mass4, (const double2*)a, (double2*)b, nrhs, DDWC_K_DSLASH64,
                              ddwc_dslash_bytes(C, nrhs, DDWC_FP64));
        launch_export<double>(ex, g, (const double2*)b, out, nrhs, MASK_ALL);
    } else if (nrhs > 1 && nrhs <= WG && ri_fits((unsigned)g.V, nrhs)) {
        // several RHS: RHS-innermost fields, the RHS of a site share its links and clover
        // (the schedule's operator workgroup size; its dispatch order only where the order table
        // may be built: the per-site arithmetic, and so the result, is the same in any order)
        const int* order = nullptr;
        const int nt = C->opt_op_threads;
        if (may_allocate && g.eo && C->opt_tile_order == 1)
            CK(tile_order(C, (unsigned)g.V, nrhs, nrhs <= nt ? nt : WG, &order, g.Vb));
        launch_import_ri32(ex, g, in, (float4*)a, nrhs);
        launch_dslash_ri32(ex, g, C->U32s, C->K32, mass4, (const float4*)a, (float4*)b, nrhs, DDWC_K_DSLASH32,
                           ddwc_dslash_bytes(C, nrhs, DDWC_MIXED32), nt, order);
        launch_export_ri32(ex, g, (const float4*)b, out, nrhs);
    } else {
        launch_import<float>(ex, g, in, (float4*)a, nrhs, MASK_ALL);
        launch_dslash<float>(ex, g, C->U32, C->K32, mass4, (const float4*)a, (float4*)b, nrhs, DDWC_K_DSLASH32,
                             ddwc_dslash_bytes(C, nrhs, DDWC_MIXED32));
        launch_export<float>(ex, g, (const float4*)b, out, nrhs, MASK_ALL);
    }
    HC(hipGetLastError());
    return DDWC_OK;
}

extern "C" int ddwc_dslash_apply(ddwc_ctx* C, double kappa, const void* in, void* out, int nrhs, int prec,
                                 void* stream) {
    CK(check_common(C, kappa, nrhs, prec));
    if (!in || !out) return fail(DDWC_EINVAL, "null vector");
    Exec ex = make_exec(C, stream);
    const bool fp64 = prec == DDWC_FP64;
    void *a, *b;
    CK(ws_get(C, fp64 ? "d_in64" : "d_in32", dslash_field_bytes(C, nrhs, prec), &a));
    CK(ws_get(C, fp64 ? "d_out64" : "d_out32", dslash_field_bytes(C, nrhs, prec), &b));
    return dslash_apply_with(C, ex, kappa, in, out, nrhs, prec, a, b, true);
}

extern "C" int ddwc_dslash_apply_noalloc(ddwc_ctx* C, double kappa, const void* in, void* out, int nrhs, int prec,
                                         void* stream) {
    CK(check_common(C, kappa, nrhs, prec));
    if (!in || !out) return fail(DDWC_EINVAL, "null vector");
    const size_t fb = (dslash_field_bytes(C, nrhs, prec) + 255) / 256 * 256;
    if (2 * fb > NOALLOC_SCRATCH_BYTES)
        return fail(DDWC_EINVAL, "ddwc_dslash_apply_noalloc: the two internal fields need " + std::to_string(2 * fb) +
                                     " bytes, more than the static scratch of " +
                                     std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes");
    if (!C->scratch) return fail(DDWC_EHIP, "no static scratch on this context's device");
    Exec ex = make_exec(C, stream);
    ex.prof = nullptr;  // no event pairs: nothing is created during the call
    char* base = (char*)C->scratch;
    return dslash_apply_with(C, ex, kappa, in, out, nrhs, prec, base, base + fb, false);
}

extern "C" int ddwc_block_solve(ddwc_ctx* C, int colour, double kappa, const void* rhs, void* sol, int nrhs,
                                double tol, int maxit, int prec, ddwc_stats* stats, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    CK(check_common(C, kappa, nrhs, prec));
    if (!rhs || !sol) return fail(DDWC_EINVAL, "null vector");
    if (colour != DDWC_BLACK && colour != DDWC_WHITE) return fail(DDWC_EINVAL, "colour must be 0 or 1");
    if (!(tol > 0) || maxit < 1) return fail(DDWC_EINVAL, "tol must be > 0 and maxit >= 1");
    Exec ex = make_exec(C, stream);
    double2 *b, *x;
    CK(ws_t(C, "api_a", vec_words(C, nrhs, true), &b));
    CK(ws_t(C, "api_b", vec_words(C, nrhs, true), &x));
    launch_import<double>(ex, C->g, rhs, b, nrhs, colour == 0 ? MASK_BLACK : MASK_WHITE);
    BlockInfo bi;
    int st = block_internal(C, ex, colour, mass_of(kappa), b, x, nrhs, tol, maxit, prec, &bi);
    if (st == DDWC_OK || st == DDWC_ENOCONV) {
        launch_export<double>(ex, C->g, x, sol, nrhs, colour == 0 ? MASK_BLACK : MASK_WHITE);
        HC(hipStreamSynchronize(ex.stream));
    }
    fill_stats(stats, bi.outer, bi.inner, bi.relres, t0);
    return st;
}

extern "C" int ddwc_solve(ddwc_ctx* C, double kappa, const void* b, void* x, int nrhs, double tol, int maxit,
                          int prec, ddwc_stats* stats, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    CK(check_common(C, kappa, nrhs, prec));
    CK(check_h16_global(C, nrhs, prec));
    if (!b || !x) return fail(DDWC_EINVAL, "null vector");
    if (!(tol > 0) || maxit < 1) return fail(DDWC_EINVAL, "tol must be > 0 and maxit >= 1");
    Exec ex = make_exec(C, stream);
    double2 *bi, *xi;
    CK(ws_t(C, "api_a", vec_words(C, nrhs, true), &bi));
    CK(ws_t(C, "api_b", vec_words(C, nrhs, true), &xi));
    launch_import<double>(ex, C->g, b, bi, nrhs, MASK_ALL);
    SolveInfo si;
    int st = solve_internal(C, ex, mass_of(kappa), bi, xi, nrhs, tol, maxit, prec, &si);
    if (st == DDWC_OK || st == DDWC_ENOCONV) {
        launch_export<double>(ex, C->g, xi, x, nrhs, MASK_ALL);
        HC(hipStreamSynchronize(ex.stream));
    }
    fill_stats(stats, si.outer, si.inner, si.relres, t0);
    return st;
}

// ------------------------------------------------------------------ SAP-preconditioned GCR
// The global solve preconditioned by the Schwarz blocks themselves (the Schwarz alternating
// procedure the paper's DD references use): M_sap eta runs NCY multiplicative cycles, each
// an approximate solve on all black blocks, a residual update, an approximate solve on all
// white blocks and a residual update, the block solves by the persistent block solver to a
// loose relative tolerance.  Flexible GCR with NKV directions per cycle, modified
// Gram-Schmidt, all in FP64 with per-RHS coefficients; the residual is recomputed exactly
// at every restart.
static int cdots(ddwc_ctx* C, Exec& ex, const double2* x, const double2* y, int nrhs, std::vector<cx<double>>& xy,
                 std::vector<double>& yy) {
    const int nt = tiles_of(C->g.V);
    double *part, *sums;
    CK(ws_t(C, "sg_part", (size_t)nt * nrhs * NPART, &part));
    CK(ws_t(C, "sg_sums", (size_t)nrhs * NPART, &sums));
    launch_dots(ex, C->g, x, y, part, nrhs);
    launch_finalize(ex, part, nt, nrhs, sums, nullptr, ST_SUM, nullptr);
    std::vector<double> h((size_t)nrhs * NPART);
    HC(hipMemcpyAsync(h.data(), sums, sizeof(double) * h.size(), hipMemcpyDeviceToHost, ex.stream));
    HC(hipStreamSynchronize(ex.stream));
    xy.resize(nrhs);
    yy.resize(nrhs);
    for (int j = 0; j < nrhs; ++j) {
        xy[j] = mk(h[(size_t)j * NPART], h[(size_t)j * NPART + 1]);
        yy[j] = h[(size_t)j * NPART + 2];
    }
    return DDWC_OK;
}

static int sap_gcr(ddwc_ctx* C, Exec& ex, double mass, const double2* b64, double2* x64, int nrhs, double tol,
                   int maxit, int prec, SolveInfo* info) {
    const int NKV = 8, NCY = 3;
    const double btol = 0.1;  // relative residual of the approximate block solves
    const Geom& g = C->g;
    const size_t nw = vec_words(C, nrhs, true);
    const double mass4 = 4.0 + mass;
    const double dbytes = ddwc_dslash_bytes(C, nrhs, DDWC_FP64);
    double2 *r, *rho, *dl, *cd;
    double* part;
    CK(ws_t(C, "sg_r", nw, &r));
    CK(ws_t(C, "sg_rho", nw, &rho));
    CK(ws_t(C, "sg_dl", nw, &dl));
    CK(ws_t(C, "sg_c", (size_t)nrhs, &cd));
    CK(ws_t(C, "sg_rpart", (size_t)tiles_of(g.V) * nrhs * NPART, &part));
    std::vector<double2*> Z(NKV), W(NKV);
    for (int k = 0; k < NKV; ++k) {
        CK(ws_t(C, "sg_z" + std::to_string(k), nw, &Z[k]));
        CK(ws_t(C, "sg_w" + std::to_string(k), nw, &W[k]));
    }
    std::vector<double2> hc(nrhs);
    auto caxpy = [&](const std::vector<cx<double>>& c, const double2* xv, double2* yv) -> int {
        for (int j = 0; j < nrhs; ++j) hc[j] = make_double2(c[j].re, c[j].im);
        HC(hipMemcpyAsync(cd, hc.data(), sizeof(double2) * nrhs, hipMemcpyHostToDevice, ex.stream));
        launch_caxpy(ex, g, cd, xv, yv, nrhs);
        HC(hipStreamSynchronize(ex.stream));  // hc is reused by the next call
        return DDWC_OK;
    };
    BlockInfo bi;
    // out = M_sap eta
    auto sap = [&](const double2* eta, double2* out) -> int {
        HC(hipMemsetAsync(out, 0, sizeof(double2) * nw, ex.stream));
        launch_axpby(ex, g, 1.0, eta, 0.0, nullptr, rho, nrhs, MASK_ALL);
        for (int cy = 0; cy < NCY; ++cy)
            for (int colour = 0; colour < 2; ++colour) {
                const int st = block_internal(C, ex, colour, mass, rho, dl, nrhs, btol, 1000, prec, &bi);
                if (st != DDWC_OK && st != DDWC_ENOCONV) return st;
                launch_axpby(ex, g, 1.0, out, 1.0, dl, out, nrhs, MASK_ALL);
                launch_residual<double>(ex, g, C->U64, C->K64, mass4, out, eta, rho, part, nrhs, DDWC_K_DSLASH64,
                                        dbytes);
            }
        return DDWC_OK;
    };
    std::vector<cx<double>> xy;
    std::vector<double> bb, rr, yy;
    CK(cdots(C, ex, b64, b64, nrhs, xy, bb));
    for (int j = 0; j < nrhs; ++j)
        if (!isfinite(bb[j])) return fail(DDWC_ENONFINITE, "non-finite right-hand side");
    HC(hipMemsetAsync(x64, 0, sizeof(double2) * nw, ex.stream));
    HC(hipMemcpyAsync(r, b64, sizeof(double2) * nw, hipMemcpyDeviceToDevice, ex.stream));
    rr = bb;
    int total = 0, nout = 0;
    bool converged = false;
    auto done = [&](int j, double rj) { return !(bb[j] > 0 && rj > tol * tol * bb[j]); };
    // a[i][k*nrhs + j]: component of w_i (normalised) in D z_k; nk, ck per (k, RHS)
    std::vector<std::vector<cx<double>>> a(NKV, std::vector<cx<double>>((size_t)NKV * nrhs));
    std::vector<double> nk((size_t)NKV * nrhs);
    std::vector<cx<double>> ck((size_t)NKV * nrhs), coef(nrhs);
    while (true) {
        bool all = true;
        for (int j = 0; j < nrhs; ++j) all = all && done(j, rr[j]);
        if (all) {
            converged = true;
            break;
        }
        if (total >= maxit || nout >= 200) break;
        ++nout;
        std::vector<double> rest = rr;
        int kused = 0;
        for (int k = 0; k < NKV && total < maxit; ++k) {
            CK(sap(r, Z[k]));
            launch_dslash<double>(ex, g, C->U64, C->K64, mass4, Z[k], W[k], nrhs, DDWC_K_DSLASH64, dbytes);
            for (int i = 0; i < k; ++i) {  // modified Gram-Schmidt
                CK(cdots(C, ex, W[i], W[k], nrhs, xy, yy));
                for (int j = 0; j < nrhs; ++j) {
                    a[i][(size_t)k * nrhs + j] = xy[j];
                    coef[j] = mk(-xy[j].re, -xy[j].im);
                }
                CK(caxpy(coef, W[i], W[k]));
            }
            CK(cdots(C, ex, W[k], W[k], nrhs, xy, yy));
            for (int j = 0; j < nrhs; ++j) {
                const double n = yy[j] > 0 ? sqrt(yy[j]) : 0.0;
                nk[(size_t)k * nrhs + j] = n;
                coef[j] = mk(n > 0 ? 1.0 / n - 1.0 : -1.0, 0.0);  // w_k <- w_k / n_k
            }
            CK(caxpy(coef, W[k], W[k]));
            CK(cdots(C, ex, W[k], r, nrhs, xy, yy));
            for (int j = 0; j < nrhs; ++j) {
                const bool use = nk[(size_t)k * nrhs + j] > 0;
                ck[(size_t)k * nrhs + j] = use ? xy[j] : mk(0.0, 0.0);
                coef[j] = use ? mk(-xy[j].re, -xy[j].im) : mk(0.0, 0.0);
                if (use) rest[j] = fmax(rest[j] - (xy[j].re * xy[j].re + xy[j].im * xy[j].im), 0.0);
            }
            CK(caxpy(coef, W[k], r));
            ++total;
            kused = k + 1;
            bool est = true;
            for (int j = 0; j < nrhs; ++j) est = est && done(j, 4.0 * rest[j]);
            if (est) break;
        }
        // x += sum_k beta_k z_k with beta from the triangular system n_k beta_k + sum_{i>k} a_ki beta_i = c_k
        std::vector<cx<double>> beta((size_t)kused * nrhs);
        for (int j = 0; j < nrhs; ++j)
            for (int k = kused - 1; k >= 0; --k) {
                const double n = nk[(size_t)k * nrhs + j];
                cx<double> t = ck[(size_t)k * nrhs + j];
                for (int i = k + 1; i < kused; ++i) t = t - a[k][(size_t)i * nrhs + j] * beta[(size_t)i * nrhs + j];
                beta[(size_t)k * nrhs + j] = n > 0 ? mk(t.re / n, t.im / n) : mk(0.0, 0.0);
            }
        for (int k = 0; k < kused; ++k) {
            for (int j = 0; j < nrhs; ++j) coef[j] = beta[(size_t)k * nrhs + j];
            CK(caxpy(coef, Z[k], x64));
        }
        // exact residual
        launch_residual<double>(ex, g, C->U64, C->K64, mass4, x64, b64, r, part, nrhs, DDWC_K_DSLASH64, dbytes);
        CK(cdots(C, ex, r, r, nrhs, xy, rr));
        for (int j = 0; j < nrhs; ++j)
            if (!isfinite(rr[j])) return fail(DDWC_ENONFINITE, "non-finite residual in the global solve");
    }
    double worst = 0;
    for (int j = 0; j < nrhs; ++j)
        if (bb[j] > 0) worst = fmax(worst, sqrt(rr[j] / bb[j]));
    if (info) {
        info->outer += nout;
        info->inner += total;
        info->relres = fmax(info->relres, worst);
    }
    if (!converged) return fail(DDWC_ENOCONV, "global solve did not reach its tolerance within maxit");
    return DDWC_OK;
}

// Dhat_P(m) e for e already projected (internal FP64): out = e - P D_bb^-1 D_bw D_ww^-1 D_wb e.
static int schur_hat(ddwc_ctx* C, Exec& ex, double mass, const double2* e, double2* out, int nrhs, double tol,
                     int prec, BlockInfo* bi) {
    const size_t nw = vec_words(C, nrhs, true);
    double2 *a, *w;
    CK(ws_t(C, "s_a", nw, &a));
    CK(ws_t(C, "s_w", nw, &w));
    // (each hop output feeds only the block solves of its colour)
    launch_hop<double>(ex, C->g, C->U64, e, a, nrhs, 1, nullptr, -1, false);
    CK(block_internal(C, ex, 1, mass, a, w, nrhs, tol, 5000, prec, bi));
    launch_hop<double>(ex, C->g, C->U64, w, a, nrhs, 0, nullptr, -1, false);
    CK(block_internal(C, ex, 0, mass, a, w, nrhs, tol, 5000, prec, bi));
    launch_axpby(ex, C->g, 1.0, e, -1.0, w, out, nrhs, MASK_P);
    return DDWC_OK;
}

// Dhat_P(m)^-1 f for f already projected: out = f - P [D^-1 (0_b, D_wb f)]_b.
static int schur_hat_inverse(ddwc_ctx* C, Exec& ex, double mass, const double2* f, double2* out, int nrhs,
                             double tol, int prec, SolveInfo* si) {
    const size_t nw = vec_words(C, nrhs, true);
    double2 *a, *chi;
    CK(ws_t(C, "s_src", nw, &a));
    CK(ws_t(C, "s_chi", nw, &chi));
    launch_hop<double>(ex, C->g, C->U64, f, a, nrhs, 1);
    CK(solve_internal(C, ex, mass, a, chi, nrhs, tol, 5000, prec, si));
    launch_axpby(ex, C->g, 1.0, f, -1.0, chi, out, nrhs, MASK_P);
    return DDWC_OK;
}

extern "C" int ddwc_schur_apply(ddwc_ctx* C, double kappa, int inverse, const void* in, void* out, int nrhs,
                                double tol, int prec, ddwc_stats* stats, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    CK(check_common(C, kappa, nrhs, prec));
    if (!in || !out) return fail(DDWC_EINVAL, "null vector");
    if (inverse != 0 && inverse != 1) return fail(DDWC_EINVAL, "inverse must be 0 or 1");
    if (inverse) CK(check_h16_global(C, nrhs, prec));
    if (!(tol > 0)) return fail(DDWC_EINVAL, "tol must be > 0");
    Exec ex = make_exec(C, stream);
    double2 *e, *o;
    CK(ws_t(C, "api_a", vec_words(C, nrhs, true), &e));
    CK(ws_t(C, "api_b", vec_words(C, nrhs, true), &o));
    launch_import<double>(ex, C->g, in, e, nrhs, MASK_P);
    int st;
    int outer = 0, inner = 0;
    double rel = 0;
    if (inverse == 0) {
        BlockInfo bi;
        st = schur_hat(C, ex, mass_of(kappa), e, o, nrhs, tol, prec, &bi);
        outer = bi.outer, inner = bi.inner, rel = bi.relres;
    } else {
        SolveInfo si;
        st = schur_hat_inverse(C, ex, mass_of(kappa), e, o, nrhs, tol, prec, &si);
        outer = si.outer, inner = si.inner, rel = si.relres;
    }
    if (st == DDWC_OK) {
        launch_export<double>(ex, C->g, o, out, nrhs, MASK_ALL);
        HC(hipStreamSynchronize(ex.stream));
    }
    fill_stats(stats, outer, inner, rel, t0);
    return st;
}

// x_i = dm P [D_bb(mp)^-1 D_bb(mn)^-1 D_bw D_ww(mp)^-1 + D_bb(mn)^-1 D_bw D_ww(mp)^-1 D_ww(mn)^-1] D_wb e
// = (Dhat_P(mp) - Dhat_P(mn)) e for e on range(P), dm = mp - mn (the resolvent difference of
// the block operators, whose masses are pure shifts).  With a region, the hops are cut to the
// outer blocks of one colour: the same expression for the Dirichlet operator of those blocks
// split by this context's blocks (nested domain decomposition).
struct Region {
    Ext4 Bo;
    int colour;
};
static int schur_diff_source(ddwc_ctx* C, Exec& ex, double mp, double mn, const double2* E, double2* G, int nrhs,
                             double tol, int prec, BlockInfo* bi, const Region* rg) {
    const Geom& g = C->g;
    const size_t nw = vec_words(C, nrhs, true);
    double2 *A, *W1, *W12, *A1;
    CK(ws_t(C, "e_A", nw, &A));
    CK(ws_t(C, "e_W1", nw, &W1));
    CK(ws_t(C, "e_W12", nw, &W12));
    CK(ws_t(C, "e_A1", nw, &A1));
    // each hop output feeds only the block solves of its colour (and the black-masked sum)
    auto hop = [&](const double2* in, double2* out, int dir) {
        launch_hop<double>(ex, g, C->U64, in, out, nrhs, dir, rg ? &rg->Bo : nullptr, rg ? rg->colour : -1, false);
    };
    hop(E, A, 1);
    CK(block_internal(C, ex, 1, mp, A, W1, nrhs, tol, 5000, prec, bi));
    CK(block_internal(C, ex, 1, mn, W1, W12, nrhs, tol, 5000, prec, bi));
    hop(W1, A, 0);
    CK(block_internal(C, ex, 0, mp, A, A1, nrhs, tol, 5000, prec, bi));
    hop(W12, A, 0);
    launch_axpby(ex, g, 1.0, A1, 1.0, A, A, nrhs, MASK_BLACK);
    CK(block_internal(C, ex, 0, mn, A, G, nrhs, tol, 5000, prec, bi));
    launch_axpby(ex, g, mp - mn, G, 0.0, nullptr, G, nrhs, MASK_P);
    return DDWC_OK;
}

// The exponents of one step from the per-RHS sums (Re<e, y>, Im<e, y>, ||y||^2) of y = M e - e:
// two flavours x = ca Re<e, y> + cb ||y||^2, one flavour x = f1 <e, y> (complex pairs).
static int store_exponents(const std::vector<double>& hs, int nrhs, int n_f, double ca, double cb, double f1,
                           double* x_row) {
    for (int j = 0; j < nrhs; ++j) {
        const double dre = hs[j * NPART], dim = hs[j * NPART + 1], nz = hs[j * NPART + 2];
        if (n_f == 2) {
            const double x = ca * dre + cb * nz;
            if (!isfinite(x)) return fail(DDWC_ENONFINITE, "non-finite exponent");
            x_row[j] = x;
        } else {
            const double xr = f1 * dre, xi = f1 * dim;
            if (!isfinite(xr) || !isfinite(xi)) return fail(DDWC_ENONFINITE, "non-finite exponent");
            x_row[2 * j] = xr;
            x_row[2 * j + 1] = xi;
        }
    }
    return DDWC_OK;
}

// log W = sum_i log W_i from the exponents x [n_interp][nrhs] (complex pairs for one flavour), and
// the per-step variances.
static int combine_steps(const double* x_host, int n_interp, int nrhs, int n_f, double* log_w,
                         double* step_var_host) {
    // Per step, with a = -Re x and a_max = max_j a_j, the weights w_j = Re exp(-x_j + a_max)
    // = exp(a_j - a_max) cos(Im x_j) (cos = 1 for two flavours): log W_i = a_max + ln sum_j w_j
    // - ln n_hit, and the step variance is var_j(w)/mean_j(w)^2.
    double lw = 0;
    bool undefined = false;
    std::vector<double> a(nrhs), w(nrhs);
    for (int i = 0; i < n_interp; ++i) {
        for (int j = 0; j < nrhs; ++j)
            a[j] = n_f == 2 ? -x_host[(size_t)i * nrhs + j] : -x_host[2 * ((size_t)i * nrhs + j)];
        double amax = a[0];
        for (int j = 1; j < nrhs; ++j) amax = fmax(amax, a[j]);
        double sw = 0, sw2 = 0;
        for (int j = 0; j < nrhs; ++j) {
            w[j] = exp(a[j] - amax);
            if (n_f == 1) w[j] *= cos(x_host[2 * ((size_t)i * nrhs + j) + 1]);
            sw += w[j];
        }
        const double mean = sw / nrhs;
        for (int j = 0; j < nrhs; ++j) sw2 += (w[j] - mean) * (w[j] - mean);
        if (!(sw > 0)) undefined = true;  // one flavour: the real part of the step mean is not positive
        lw += amax + log(sw) - log((double)nrhs);
        const double var = nrhs > 1 ? (sw2 / (nrhs - 1)) / (mean * mean) : 0.0;
        if (!isfinite(var)) undefined = true;
        if (step_var_host) step_var_host[i] = var;
    }
    *log_w = undefined ? NAN : lw;
    if (!isfinite(lw) || undefined)
        return fail(DDWC_EUNDEF, "estimate undefined (non-positive real step mean, or non-finite mean or variance)");
    return DDWC_OK;
}

extern "C" int ddwc_log_w_combine(const double* x_host, int n_interp, int n_hit, int n_f, double* log_w,
                                  double* step_var_host, double* gx_host) {
    if (!x_host || !log_w) return fail(DDWC_EINVAL, "null argument");
    if (n_interp < 1 || n_interp > 4096) return fail(DDWC_EINVAL, "n_interp must be in [1, 4096]");
    if (n_hit < 1 || n_hit > 65535) return fail(DDWC_EINVAL, "n_hit must be in [1, 65535]");
    if (n_f != 1 && n_f != 2) return fail(DDWC_EINVAL, "n_f must be 1 or 2");
    if (gx_host && n_f != 2) return fail(DDWC_EINVAL, "the gradient is defined for two flavours only");
    const size_t nx = (size_t)n_interp * n_hit * (n_f == 2 ? 1 : 2);
    for (size_t k = 0; k < nx; ++k)
        if (!isfinite(x_host[k])) return fail(DDWC_EINVAL, "non-finite exponent");
    if (gx_host) {
        // d log W_i / d x_ij = -exp(-x_ij) / sum_j exp(-x_ij), formed relative to the step's largest -x
        for (int i = 0; i < n_interp; ++i) {
            const double* x = x_host + (size_t)i * n_hit;
            double amax = -x[0];
            for (int j = 1; j < n_hit; ++j) amax = fmax(amax, -x[j]);
            double sw = 0;
            for (int j = 0; j < n_hit; ++j) sw += exp(-x[j] - amax);
            for (int j = 0; j < n_hit; ++j) gx_host[(size_t)i * n_hit + j] = -exp(-x[j] - amax) / sw;
        }
    }
    return combine_steps(x_host, n_interp, n_hit, n_f, log_w, step_var_host);
}

extern "C" int ddwc_det_ratio_estimate(ddwc_ctx* C, double kappa1, double kappa2, int n_interp, int op, int n_f,
                                       const void* eta, int n_hit, double tol, int prec, double* x_host,
                                       double* log_w_gl, double* step_var_host, ddwc_stats* stats, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    CK(check_common(C, kappa1, n_hit, prec));
    CK(check_h16_global(C, n_hit, prec));
    if (!(kappa2 > 0) || !isfinite(kappa2)) return fail(DDWC_EINVAL, "kappa2 must be positive and finite");
    if (n_interp < 1 || n_interp > 4096) return fail(DDWC_EINVAL, "n_interp must be in [1, 4096]");
    if (op != DDWC_OP_FULL && op != DDWC_OP_SCHUR) return fail(DDWC_EINVAL, "op must be FULL (0) or SCHUR (1)");
    if (n_f != 1 && n_f != 2) return fail(DDWC_EINVAL, "n_f must be 1 or 2");
    if (!eta || !x_host || !log_w_gl) return fail(DDWC_EINVAL, "null argument");
    if (!(tol > 0)) return fail(DDWC_EINVAL, "tol must be > 0");
    Exec ex = make_exec(C, stream);
    const Geom& g = C->g;
    const int nrhs = n_hit;
    const size_t nw = vec_words(C, nrhs, true);
    const int nt = tiles_of(g.V);
    const double m1 = mass_of(kappa1), m2 = mass_of(kappa2);
    double2 *E, *G, *Z;
    double *part, *sums;
    CK(ws_t(C, "e_E", nw, &E));
    CK(ws_t(C, "e_G", nw, &G));
    CK(ws_t(C, "e_Z", nw, &Z));
    CK(ws_t(C, "e_part", (size_t)nt * nrhs * NPART, &part));
    CK(ws_t(C, "e_sums", (size_t)nrhs * NPART, &sums));
    SolveInfo si;
    BlockInfo bi;
    std::vector<double> hs((size_t)nrhs * NPART);
    for (int i = 0; i < n_interp; ++i) {
        // m_i = (i/N) m2 + ((N - i)/N) m1
        const double mp = ((double)i / n_interp) * m2 + ((double)(n_interp - i) / n_interp) * m1;
        const double mn = ((double)(i + 1) / n_interp) * m2 + ((double)(n_interp - i - 1) / n_interp) * m1;
        const double dm = mp - mn;
        const char* eta_i = (const char*)eta + (size_t)i * nrhs * g.V * 12 * 16;
        double ca, cb;  // x = ca * Re<e, y> + cb * ||y||^2
        if (op == DDWC_OP_FULL) {
            // M eta - eta = dm D(mn)^-1 eta
            launch_import<double>(ex, g, eta_i, E, nrhs, MASK_ALL);
            CK(solve_internal(C, ex, mn, E, Z, nrhs, tol, 5000, prec, &si));
            ca = 2 * dm;
            cb = dm * dm;
        } else {
            // Mh eta - eta = Dhat(mn)^-1 g, g = dm P [D_bb(mp)^-1 D_bb(mn)^-1 D_bw D_ww(mp)^-1
            //                + D_bb(mn)^-1 D_bw D_ww(mp)^-1 D_ww(mn)^-1] D_wb eta
            launch_import<double>(ex, g, eta_i, E, nrhs, MASK_P);
            CK(schur_diff_source(C, ex, mp, mn, E, G, nrhs, tol, prec, &bi, nullptr));
            CK(schur_hat_inverse(C, ex, mn, G, Z, nrhs, tol, prec, &si));
            ca = 2.0;
            cb = 1.0;
        }
        launch_dots(ex, g, E, Z, part, nrhs);
        launch_finalize(ex, part, nt, nrhs, sums, nullptr, ST_SUM, nullptr);
        HC(hipMemcpyAsync(hs.data(), sums, sizeof(double) * nrhs * NPART, hipMemcpyDeviceToHost, ex.stream));
        HC(hipStreamSynchronize(ex.stream));
        // one flavour: x = eta^+ (M - 1) eta = <eta, y> with y = M eta - eta: dm <eta, psi> or <e, zeta>
        CK(store_exponents(hs, nrhs, n_f, ca, cb, op == DDWC_OP_FULL ? dm : 1.0,
                           x_host + (size_t)i * nrhs * (n_f == 2 ? 1 : 2)));
    }
    *log_w_gl = NAN;
    fill_stats(stats, si.outer, si.inner, si.relres, t0);
    return combine_steps(x_host, n_interp, nrhs, n_f, log_w_gl, step_var_host);
}

// Nested domain decomposition (Sec. 2.2): for the outer blocks of one colour, A = D_cc split by
// the inner context's blocks, Ahat = 1 - A_bb^-1 A_bw A_ww^-1 A_wb on range(P_c), P_c the black
// inner face sites inside those outer blocks.  Per step, Mh e - e = Ahat(mn)^-1 g with g from
// schur_diff_source (hops cut to the region), and Ahat(mn)^-1 g = g - P_c [A(mn)^-1 (0, A_wb g)]_b,
// the inversion of A being the outer context's block solve of that colour.
extern "C" int ddwc_det_ratio_nested(ddwc_ctx* O, ddwc_ctx* I, int colour, double kappa1, double kappa2,
                                     int n_interp, int n_f, const void* eta, int n_hit, double tol, int prec,
                                     double* x_host, double* log_w, double* step_var_host, ddwc_stats* stats,
                                     void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    CK(check_common(I, kappa1, n_hit, prec));
    CK(check_common(O, kappa1, n_hit, prec));
    if (O == I) return fail(DDWC_EINVAL, "outer and inner must be different contexts");
    for (int mu = 0; mu < 4; ++mu) {
        if (O->lat[mu] != I->lat[mu]) return fail(DDWC_EINVAL, "outer and inner contexts differ in lattice size");
        if (O->blk[mu] % I->blk[mu] != 0)
            return fail(DDWC_EINVAL, "inner block extents must divide the outer block extents");
    }
    if (O->g.tbc != I->g.tbc || O->csw != I->csw || O->links_fp != I->links_fp)
        return fail(DDWC_EINVAL, "outer and inner contexts differ in links, c_sw or time boundary");
    if (colour != 0 && colour != 1) return fail(DDWC_EINVAL, "colour must be 0 or 1");
    if (!(kappa2 > 0) || !isfinite(kappa2)) return fail(DDWC_EINVAL, "kappa2 must be positive and finite");
    if (n_interp < 1 || n_interp > 4096) return fail(DDWC_EINVAL, "n_interp must be in [1, 4096]");
    if (n_f != 1 && n_f != 2) return fail(DDWC_EINVAL, "n_f must be 1 or 2");
    if (!eta || !x_host || !log_w) return fail(DDWC_EINVAL, "null argument");
    if (!(tol > 0)) return fail(DDWC_EINVAL, "tol must be > 0");
    Exec ex = make_exec(I, stream), exo = make_exec(O, stream);
    const Geom& g = I->g;
    const int nrhs = n_hit;
    const size_t nw = vec_words(I, nrhs, true);
    const int nt = tiles_of(g.V);
    const double m1 = mass_of(kappa1), m2 = mass_of(kappa2);
    Region rg;
    for (int mu = 0; mu < 4; ++mu) rg.Bo.v[mu] = O->blk[mu];
    rg.colour = colour;
    double2 *E, *G, *Z, *S, *So, *Xo;
    double *part, *sums;
    CK(ws_t(I, "e_E", nw, &E));
    CK(ws_t(I, "e_G", nw, &G));
    CK(ws_t(I, "e_Z", nw, &Z));
    CK(ws_t(I, "n_S", nw, &S));
    CK(ws_t(O, "n_So", nw, &So));
    CK(ws_t(O, "n_Xo", nw, &Xo));
    CK(ws_t(I, "e_part", (size_t)nt * nrhs * NPART, &part));
    CK(ws_t(I, "e_sums", (size_t)nrhs * NPART, &sums));
    BlockInfo bi, bo;
    std::vector<double> hs((size_t)nrhs * NPART);
    for (int i = 0; i < n_interp; ++i) {
        const double mp = ((double)i / n_interp) * m2 + ((double)(n_interp - i) / n_interp) * m1;
        const double mn = ((double)(i + 1) / n_interp) * m2 + ((double)(n_interp - i - 1) / n_interp) * m1;
        const char* eta_i = (const char*)eta + (size_t)i * nrhs * g.V * 12 * 16;
        launch_import<double>(ex, g, eta_i, E, nrhs, MASK_P);
        launch_region(ex, g, rg.Bo, colour, E, nrhs);
        CK(schur_diff_source(I, ex, mp, mn, E, G, nrhs, tol, prec, &bi, &rg));
        // Ahat(mn)^-1 G
        launch_hop<double>(ex, g, I->U64, G, S, nrhs, 1, &rg.Bo, colour);
        launch_relayout(ex, g, O->g, S, So, nrhs);
        CK(block_internal(O, exo, colour, mn, So, Xo, nrhs, tol, 5000, prec, &bo));
        launch_relayout(ex, O->g, g, Xo, S, nrhs);
        launch_axpby(ex, g, 1.0, G, -1.0, S, Z, nrhs, MASK_P);
        launch_dots(ex, g, E, Z, part, nrhs);
        launch_finalize(ex, part, nt, nrhs, sums, nullptr, ST_SUM, nullptr);
        HC(hipMemcpyAsync(hs.data(), sums, sizeof(double) * nrhs * NPART, hipMemcpyDeviceToHost, ex.stream));
        HC(hipStreamSynchronize(ex.stream));
        CK(store_exponents(hs, nrhs, n_f, 2.0, 1.0, 1.0, x_host + (size_t)i * nrhs * (n_f == 2 ? 1 : 2)));
    }
    *log_w = NAN;
    fill_stats(stats, bo.outer, bo.inner, bo.relres, t0);
    return combine_steps(x_host, n_interp, nrhs, n_f, log_w, step_var_host);
}

// Re <x, y> per RHS, to the host.
static int redots(ddwc_ctx* C, Exec& ex, const double2* x, const double2* y, int nrhs, std::vector<double>& out) {
    const int nt = tiles_of(C->g.V);
    double *part, *sums;
    CK(ws_t(C, "gr_part", (size_t)nt * nrhs * NPART, &part));
    CK(ws_t(C, "gr_sums", (size_t)nrhs * NPART, &sums));
    launch_dots(ex, C->g, x, y, part, nrhs);
    launch_finalize(ex, part, nt, nrhs, sums, nullptr, ST_SUM, nullptr);
    std::vector<double> h((size_t)nrhs * NPART);
    HC(hipMemcpyAsync(h.data(), sums, sizeof(double) * h.size(), hipMemcpyDeviceToHost, ex.stream));
    HC(hipStreamSynchronize(ex.stream));
    out.resize(nrhs);
    for (int j = 0; j < nrhs; ++j) out[j] = h[(size_t)j * NPART];
    return DDWC_OK;
}

// Gradient of L = sum_ij gx_ij x_ij (x_ij the two-flavour exponents of ddwc_det_ratio_estimate)
// with respect to kappa2 and the links.  With y = M eta and z = D_n^-+ y (full M; D^+ = g5 D g5)
// or z = Dhat_n^-+ y (Schur):  dx = 2 Re <z, dD_p eta> - 2 Re <z, dD_n y>, and for the Schur
// form, with a = D_bb^-+ P z, c = D_ww^-+ D_bw^+ a, w1 = D_ww^-1 D_wb v, w2 = D_bb^-1 D_bw w1,
//     <z, dDhat v> = <a, dD (w2 - w1)> + <c, dD (w1 - v)>,
// so dDhat/dm gives <a, w2> + <c, w1> and the links enter through Re <a, dD b> pairs.
extern "C" int ddwc_det_ratio_grad(ddwc_ctx* C, double kappa1, double kappa2, int n_interp, int op, const void* eta,
                                   int n_hit, double tol, int prec, const double* gx, double* dkappa2, void* dU,
                                   ddwc_stats* stats, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    CK(check_common(C, kappa1, n_hit, prec));
    CK(check_h16_global(C, n_hit, prec));
    if (!(kappa2 > 0) || !isfinite(kappa2)) return fail(DDWC_EINVAL, "kappa2 must be positive and finite");
    if (n_interp < 1 || n_interp > 4096) return fail(DDWC_EINVAL, "n_interp must be in [1, 4096]");
    if (op != DDWC_OP_FULL && op != DDWC_OP_SCHUR) return fail(DDWC_EINVAL, "op must be FULL (0) or SCHUR (1)");
    if (!eta || !gx) return fail(DDWC_EINVAL, "null argument");
    if (!dkappa2 && !dU) return fail(DDWC_EINVAL, "neither dkappa2 nor dU requested");
    if (!(tol > 0)) return fail(DDWC_EINVAL, "tol must be > 0");
    for (size_t k = 0; k < (size_t)n_interp * n_hit; ++k)
        if (!isfinite(gx[k])) return fail(DDWC_EINVAL, "non-finite upstream gradient");
    Exec ex = make_exec(C, stream);
    const Geom& g = C->g;
    const int nrhs = n_hit;
    const size_t nw = vec_words(C, nrhs, true);
    const double m1 = mass_of(kappa1), m2 = mass_of(kappa2);
    double2 *E, *A, *W1, *W12, *A1, *Gs, *Z, *Y, *W1n, *W2n, *Y5, *Zh, *Ap, *Cp, *An, *Cn, *B;
    const char* nm[17] = {"gr_E", "gr_A", "gr_W1", "gr_W12", "gr_A1", "gr_G", "gr_Z", "gr_Y", "gr_W1n",
                          "gr_W2n", "gr_Y5", "gr_Zh", "gr_Ap", "gr_Cp", "gr_An", "gr_Cn", "gr_B"};
    double2** vp[17] = {&E, &A, &W1, &W12, &A1, &Gs, &Z, &Y, &W1n, &W2n, &Y5, &Zh, &Ap, &Cp, &An, &Cn, &B};
    for (int k = 0; k < 17; ++k) CK(ws_t(C, nm[k], nw, vp[k]));
    cx<double>* Gd = nullptr;
    double* wd;
    CK(ws_t(C, "gr_w", (size_t)nrhs, &wd));
    if (dU) {
        CK(ws_t(C, "gr_force", (size_t)36 * g.V, &Gd));
        HC(hipMemsetAsync(Gd, 0, (size_t)36 * g.V * sizeof(cx<double>), ex.stream));
    }
    auto force = [&](const double2* a, const double2* b, const std::vector<double>& w) -> int {
        HC(hipMemcpyAsync(wd, w.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, ex.stream));
        launch_force_hop(ex, g, C->nbr, a, b, wd, nrhs, Gd);
        if (C->csw != 0.0) launch_force_clover(ex, g, C->U64, C->csw, a, b, wd, nrhs, Gd);
        HC(hipStreamSynchronize(ex.stream));
        return DDWC_OK;
    };
    SolveInfo si;
    BlockInfo bi;
    const int MAXIT = 5000;
    double dLdm2 = 0;
    std::vector<double> d1, d2, wpos(nrhs), wneg(nrhs);
    for (int i = 0; i < n_interp; ++i) {
        const double mp = ((double)i / n_interp) * m2 + ((double)(n_interp - i) / n_interp) * m1;
        const double mn = ((double)(i + 1) / n_interp) * m2 + ((double)(n_interp - i - 1) / n_interp) * m1;
        const double dm = mp - mn, fp = (double)i / n_interp, fn = (double)(i + 1) / n_interp;  // dm_i/dm2
        const char* eta_i = (const char*)eta + (size_t)i * nrhs * g.V * 12 * 16;
        const double* gi = gx + (size_t)i * nrhs;
        for (int j = 0; j < nrhs; ++j) {
            wpos[j] = 2 * gi[j];
            wneg[j] = -2 * gi[j];
        }
        std::vector<double> dp(nrhs), dn(nrhs);
        if (op == DDWC_OP_FULL) {
            launch_import<double>(ex, g, eta_i, E, nrhs, MASK_ALL);
            CK(solve_internal(C, ex, mn, E, Z, nrhs, tol, MAXIT, prec, &si));  // psi
            launch_axpby(ex, g, 1.0, E, dm, Z, Y, nrhs, MASK_ALL);             // y = eta + dm psi
            launch_axpby(ex, g, 1.0, Y, 0.0, nullptr, Y5, nrhs, MASK_ALL);
            launch_gamma5(ex, g, Y5, nrhs);
            CK(solve_internal(C, ex, mn, Y5, Zh, nrhs, tol, MAXIT, prec, &si));
            launch_gamma5(ex, g, Zh, nrhs);  // z = D_n^-+ y
            CK(redots(C, ex, Zh, E, nrhs, d1));
            CK(redots(C, ex, Zh, Y, nrhs, d2));
            for (int j = 0; j < nrhs; ++j) {
                dp[j] = 2 * d1[j];
                dn[j] = -2 * d2[j];
            }
            if (dU) {
                launch_axpby(ex, g, 1.0, E, -1.0, Y, B, nrhs, MASK_ALL);  // eta - y
                CK(force(Zh, B, wpos));
            }
        } else {
            // forward quantities of the difference form (as in ddwc_det_ratio_estimate)
            launch_import<double>(ex, g, eta_i, E, nrhs, MASK_P);
            launch_hop<double>(ex, g, C->U64, E, A, nrhs, 1);
            CK(block_internal(C, ex, 1, mp, A, W1, nrhs, tol, MAXIT, prec, &bi));
            CK(block_internal(C, ex, 1, mn, W1, W12, nrhs, tol, MAXIT, prec, &bi));
            launch_hop<double>(ex, g, C->U64, W1, A, nrhs, 0);
            CK(block_internal(C, ex, 0, mp, A, A1, nrhs, tol, MAXIT, prec, &bi));
            launch_hop<double>(ex, g, C->U64, W12, A, nrhs, 0);
            launch_axpby(ex, g, 1.0, A1, 1.0, A, A, nrhs, MASK_BLACK);
            CK(block_internal(C, ex, 0, mn, A, Gs, nrhs, tol, MAXIT, prec, &bi));
            launch_axpby(ex, g, dm, Gs, 0.0, nullptr, Gs, nrhs, MASK_P);
            CK(schur_hat_inverse(C, ex, mn, Gs, Z, nrhs, tol, prec, &si));
            launch_axpby(ex, g, 1.0, E, 1.0, Z, Y, nrhs, MASK_P);  // y = Mhat e
            // w1, w2 for v = y at m_n (for v = e at m_p they are W1 and A1)
            launch_hop<double>(ex, g, C->U64, Y, A, nrhs, 1);
            CK(block_internal(C, ex, 1, mn, A, W1n, nrhs, tol, MAXIT, prec, &bi));
            launch_hop<double>(ex, g, C->U64, W1n, A, nrhs, 0);
            CK(block_internal(C, ex, 0, mn, A, W2n, nrhs, tol, MAXIT, prec, &bi));
            // adjoint: Dhat_P is not gamma_5-hermitian (D_bb^-1 acts from the left), but
            // Dhat_P^-+ v = v - g5 P D_bw [D^-1 (g5 v)]_w, so zh = g5 z = u - P D_bw [D_n^-1 u]_w
            // with u = g5 y; then a = g5 D_bb^-1 zh and c = g5 D_ww^-1 D_wb (g5 a)
            launch_axpby(ex, g, 1.0, Y, 0.0, nullptr, Y5, nrhs, MASK_P);
            launch_gamma5(ex, g, Y5, nrhs);
            CK(solve_internal(C, ex, mn, Y5, W12, nrhs, tol, MAXIT, prec, &si));
            launch_hop<double>(ex, g, C->U64, W12, A, nrhs, 0);
            launch_axpby(ex, g, 1.0, Y5, -1.0, A, Zh, nrhs, MASK_P);
            CK(block_internal(C, ex, 0, mp, Zh, Ap, nrhs, tol, MAXIT, prec, &bi));
            launch_hop<double>(ex, g, C->U64, Ap, A, nrhs, 1);
            CK(block_internal(C, ex, 1, mp, A, Cp, nrhs, tol, MAXIT, prec, &bi));
            CK(block_internal(C, ex, 0, mn, Zh, An, nrhs, tol, MAXIT, prec, &bi));
            launch_hop<double>(ex, g, C->U64, An, A, nrhs, 1);
            CK(block_internal(C, ex, 1, mn, A, Cn, nrhs, tol, MAXIT, prec, &bi));
            launch_gamma5(ex, g, Ap, nrhs);
            launch_gamma5(ex, g, Cp, nrhs);
            launch_gamma5(ex, g, An, nrhs);
            launch_gamma5(ex, g, Cn, nrhs);
            CK(redots(C, ex, Ap, A1, nrhs, d1));
            CK(redots(C, ex, Cp, W1, nrhs, d2));
            for (int j = 0; j < nrhs; ++j) dp[j] = 2 * (d1[j] + d2[j]);
            CK(redots(C, ex, An, W2n, nrhs, d1));
            CK(redots(C, ex, Cn, W1n, nrhs, d2));
            for (int j = 0; j < nrhs; ++j) dn[j] = -2 * (d1[j] + d2[j]);
            if (dU) {
                launch_axpby(ex, g, 1.0, A1, -1.0, W1, B, nrhs, MASK_ALL);
                CK(force(Ap, B, wpos));
                launch_axpby(ex, g, 1.0, W1, -1.0, E, B, nrhs, MASK_ALL);
                CK(force(Cp, B, wpos));
                launch_axpby(ex, g, 1.0, W2n, -1.0, W1n, B, nrhs, MASK_ALL);
                CK(force(An, B, wneg));
                launch_axpby(ex, g, 1.0, W1n, -1.0, Y, B, nrhs, MASK_ALL);
                CK(force(Cn, B, wneg));
            }
        }
        for (int j = 0; j < nrhs; ++j) dLdm2 += gi[j] * (dp[j] * fp + dn[j] * fn);
    }
    if (dkappa2) *dkappa2 = dLdm2 * (-0.5 / (kappa2 * kappa2));
    if (dU) launch_links_export(ex, g, Gd, dU);
    HC(hipStreamSynchronize(ex.stream));
    HC(hipGetLastError());
    fill_stats(stats, si.outer, si.inner, si.relres, t0);
    if (dkappa2 && !isfinite(*dkappa2)) return fail(DDWC_ENONFINITE, "non-finite derivative");
    return DDWC_OK;
}

extern "C" int ddwc_link_force(ddwc_ctx* C, const void* a, const void* b, int nrhs, const double* w_host, void* dU,
                               void* stream) {
    CK(check_ctx(C));
    if (nrhs < 1 || nrhs > 4096) return fail(DDWC_EINVAL, "nrhs must be in [1, 4096]");
    if (!a || !b || !w_host || !dU) return fail(DDWC_EINVAL, "null argument");
    for (int r = 0; r < nrhs; ++r)
        if (!isfinite(w_host[r])) return fail(DDWC_EINVAL, "non-finite weight");
    Exec ex = make_exec(C, stream);
    const Geom& g = C->g;
    double2 *ai, *bi;
    double* wd;
    cx<double>* Gd;
    CK(ws_t(C, "api_a", vec_words(C, nrhs, true), &ai));
    CK(ws_t(C, "api_b", vec_words(C, nrhs, true), &bi));
    CK(ws_t(C, "gr_w", (size_t)nrhs, &wd));
    CK(ws_t(C, "gr_force", (size_t)36 * g.V, &Gd));
    launch_import<double>(ex, g, a, ai, nrhs, MASK_ALL);
    launch_import<double>(ex, g, b, bi, nrhs, MASK_ALL);
    HC(hipMemcpyAsync(wd, w_host, sizeof(double) * nrhs, hipMemcpyHostToDevice, ex.stream));
    HC(hipMemsetAsync(Gd, 0, (size_t)36 * g.V * sizeof(cx<double>), ex.stream));
    launch_force_hop(ex, g, C->nbr, ai, bi, wd, nrhs, Gd);
    if (C->csw != 0.0) launch_force_clover(ex, g, C->U64, C->csw, ai, bi, wd, nrhs, Gd);
    launch_links_export(ex, g, Gd, dU);
    HC(hipStreamSynchronize(ex.stream));
    HC(hipGetLastError());
    return DDWC_OK;
}

extern "C" int ddwc_block_logdet(ddwc_ctx* C, double kappa, int colour, double* logabs_host, int* sign_host,
                                 void* stream) {
    CK(check_common(C, kappa, 1, DDWC_FP64));
    if (colour != DDWC_BLACK && colour != DDWC_WHITE) return fail(DDWC_EINVAL, "colour must be 0 or 1");
    if (!logabs_host) return fail(DDWC_EINVAL, "null argument");
    const Geom& g = C->g;
    const size_t n = g.eo ? (size_t)12 * g.hvb : (size_t)12 * g.Vb;
    const size_t mbytes = n * n * sizeof(cx<double>);
    const size_t budget = (size_t)16 << 30;  // device memory for one batch of dense blocks
    if (mbytes > budget) return fail(DDWC_EINVAL, "Schwarz block too large for dense block determinants");
    const int NB = g.NBc;
    const int batch = (int)std::min<size_t>((size_t)NB, std::max<size_t>(1, budget / mbytes));
    if (!C->blas && !(C->blas = blas_handle_create())) return fail(DDWC_EHIP, "dense linear-algebra handle");
    Exec ex = make_exec(C, stream);
    const double mass4 = 4.0 + mass_of(kappa);
    cx<double>* Mat;
    int *ipiv, *info;
    double *odd, *lu;
    CK(ws_t(C, "bd_mat", (size_t)batch * n * n, &Mat));
    CK(ws_t(C, "bd_ipiv", (size_t)batch * n, &ipiv));
    CK(ws_t(C, "bd_info", (size_t)batch, &info));
    CK(ws_t(C, "bd_odd", (size_t)NB, &odd));
    CK(ws_t(C, "bd_lu", (size_t)2 * NB, &lu));
    HC(hipMemsetAsync(odd, 0, NB * sizeof(double), ex.stream));
    if (g.eo) launch_bd_oddlogdet(ex, g, C->K64, mass4, colour, odd);
    std::vector<int> hinfo(batch);
    bool singular = false;
    for (int r0 = 0; r0 < NB; r0 += batch) {
        const int nb = std::min(batch, NB - r0);
        const int st = block_logdet_run(ex, g, C->U64, C->K64, C->nbr, mass4, colour, r0, nb, C->blas, Mat, ipiv,
                                        info, lu + 2 * r0);
        if (st != 0) return fail(DDWC_EHIP, "batched LU of the block matrices failed (" + std::to_string(st) + ")");
        HC(hipMemcpyAsync(hinfo.data(), info, nb * sizeof(int), hipMemcpyDeviceToHost, ex.stream));
        HC(hipStreamSynchronize(ex.stream));
        for (int b = 0; b < nb; ++b) singular |= hinfo[b] != 0;
    }
    std::vector<double> hodd(NB), hlu(2 * NB);
    HC(hipMemcpyAsync(hodd.data(), odd, NB * sizeof(double), hipMemcpyDeviceToHost, ex.stream));
    HC(hipMemcpyAsync(hlu.data(), lu, 2 * NB * sizeof(double), hipMemcpyDeviceToHost, ex.stream));
    HC(hipStreamSynchronize(ex.stream));
    HC(hipGetLastError());
    bool undefined = singular;
    for (int b = 0; b < NB; ++b) {
        logabs_host[b] = hodd[b] + hlu[2 * b];
        // det D_k is real: the phase is a multiple of pi up to rounding
        const double ph = hlu[2 * b + 1];
        const double c = cos(ph), sn = sin(ph);
        if (!isfinite(logabs_host[b]) || fabs(sn) > 1e-6) undefined = true;
        if (sign_host) sign_host[b] = c >= 0 ? 1 : -1;
    }
    if (undefined) return fail(DDWC_EUNDEF, "block determinant singular, not finite or not real");
    return DDWC_OK;
}

extern "C" int ddwc_log_w_blocks(ddwc_ctx* C, double kappa1, double kappa2, double* out_host, void* stream) {
    CK(check_common(C, kappa1, 1, DDWC_FP64));
    if (!(kappa2 > 0) || !isfinite(kappa2)) return fail(DDWC_EINVAL, "kappa2 must be positive and finite");
    if (!out_host) return fail(DDWC_EINVAL, "null argument");
    // 2 sum_k [ln|det D_k(m2)| - ln|det D_k(m1)|] over the blocks of both colours; the sums run per
    // colour and mass in block order, then in the fixed order (black m2, black m1, white m2, white m1)
    std::vector<double> la(C->g.NBc);
    double tot = 0;
    for (int c = DDWC_BLACK; c <= DDWC_WHITE; ++c)
        for (int k = 0; k < 2; ++k) {
            CK(ddwc_block_logdet(C, k == 0 ? kappa2 : kappa1, c, la.data(), nullptr, stream));
            double s = 0;
            for (double v : la) s += v;
            tot += k == 0 ? s : -s;
        }
    *out_host = 2.0 * tot;
    return DDWC_OK;
}

extern "C" int ddwc_log_w_nested_total(ddwc_ctx* O, ddwc_ctx* I, double kappa1, double kappa2, int n_interp,
                                       const void* eta_gl, int n_hit_gl, const void* eta_black,
                                       const void* eta_white, int n_hit_nested, double tol, int prec,
                                       double* parts_host, ddwc_stats* stats, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!eta_gl || !eta_black || !eta_white || !parts_host) return fail(DDWC_EINVAL, "null argument");
    if (n_interp < 1 || n_interp > 4096) return fail(DDWC_EINVAL, "n_interp must be in [1, 4096]");
    if (n_hit_gl < 1 || n_hit_gl > 65535 || n_hit_nested < 1 || n_hit_nested > 65535)
        return fail(DDWC_EINVAL, "n_hit must be in [1, 65535]");
    double parts[5] = {0, 0, 0, 0, 0};
    std::vector<double> x((size_t)n_interp * std::max(n_hit_gl, n_hit_nested));
    ddwc_stats st;
    // the nested calls check both contexts (same lattice, links, c_sw, boundary; dividing blocks) first
    const void* eta_c[2] = {eta_black, eta_white};
    for (int c = DDWC_BLACK; c <= DDWC_WHITE; ++c)
        CK(ddwc_det_ratio_nested(O, I, c, kappa1, kappa2, n_interp, 2, eta_c[c], n_hit_nested, tol, prec, x.data(),
                                 &parts[1 + c], nullptr, nullptr, stream));
    CK(ddwc_det_ratio_estimate(O, kappa1, kappa2, n_interp, DDWC_OP_SCHUR, 2, eta_gl, n_hit_gl, tol, prec, x.data(),
                               &parts[0], nullptr, &st, stream));
    CK(ddwc_log_w_blocks(I, kappa1, kappa2, &parts[3], stream));
    parts[4] = ((parts[0] + parts[1]) + parts[2]) + parts[3];
    for (int k = 0; k < 5; ++k) parts_host[k] = parts[k];
    if (stats) {
        *stats = st;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return DDWC_OK;
}

extern "C" int ddwc_set_option(ddwc_ctx* C, int option, int value) {
    CK(check_ctx(C));
    switch (option) {
        case DDWC_OPT_GRAPHS:
            if (value != 0 && value != 1) return fail(DDWC_EINVAL, "graphs option must be 0 or 1");
            C->opt_graphs = value;
            break;
        case DDWC_OPT_POLL:
            if (value < 1 || value > 64) return fail(DDWC_EINVAL, "poll interval must be in [1, 64]");
            C->opt_poll = value;
            break;
        case DDWC_OPT_BLOCK_THREADS:
            if (value != 0 && (value < 64 || value > 768 || value % 64 != 0))
                return fail(DDWC_EINVAL, "block threads must be 0 or a multiple of 64 in [64, 768]");
            C->opt_blk_threads = value;
            break;
        case DDWC_OPT_SOLVER:
            if (value != 0 && value != 1) return fail(DDWC_EINVAL, "solver must be 0 or 1");
            C->opt_solver = value;
            break;
        case DDWC_OPT_BLOCK_LDS: {
            int maxlds = 0;
            HC(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, C->device));
            if (value < 0 || ((long long)value << 10) + 1024 > maxlds)
                return fail(DDWC_EINVAL, "block LDS reservation must be in [0, " + std::to_string(maxlds / 1024 - 1) +
                                             "] KiB");
            C->opt_blk_lds = value;
            break;
        }
        case DDWC_OPT_BLOCK_KERNEL:
            if (value != 0 && value != 1) return fail(DDWC_EINVAL, "block kernel must be 0 or 1");
            C->opt_blk_kernel = value;
            break;
        case DDWC_OPT_INNER_FLOOR:
            if (value < 1 || value > 100000) return fail(DDWC_EINVAL, "inner floor must be in [1, 100000] (x 1e-8)");
            C->opt_inner_floor = value;
            break;
        case DDWC_OPT_OP_THREADS:
            if (value != 128 && value != 256 && value != 512)
                return fail(DDWC_EINVAL, "operator threads must be 128, 256 or 512");
            C->opt_op_threads = value;
            break;
        case DDWC_OPT_TILE_ORDER:
            if (value != 0 && value != 1) return fail(DDWC_EINVAL, "tile order must be 0 or 1");
            C->opt_tile_order = value;
            break;
        default:
            return fail(DDWC_EINVAL, "unknown option");
    }
    return DDWC_OK;
}

extern "C" int ddwc_get_option(ddwc_ctx* C, int option, int* value) {
    CK(check_ctx(C));
    if (!value) return fail(DDWC_EINVAL, "null argument");
    switch (option) {
        case DDWC_OPT_GRAPHS: *value = C->opt_graphs; break;
        case DDWC_OPT_POLL: *value = C->opt_poll; break;
        case DDWC_OPT_BLOCK_THREADS: *value = C->opt_blk_threads; break;
        case DDWC_OPT_SOLVER: *value = C->opt_solver; break;
        case DDWC_OPT_BLOCK_LDS: *value = C->opt_blk_lds; break;
        case DDWC_OPT_BLOCK_KERNEL: *value = C->opt_blk_kernel; break;
        case DDWC_OPT_INNER_FLOOR: *value = C->opt_inner_floor; break;
        case DDWC_OPT_OP_THREADS: *value = C->opt_op_threads; break;
        case DDWC_OPT_TILE_ORDER: *value = C->opt_tile_order; break;
        default: return fail(DDWC_EINVAL, "unknown option");
    }
    return DDWC_OK;
}

// Times the schedule choices on this context's lattice with nrhs reproducible right-hand
// sides and keeps the fastest, one group after the other: the block inner solver (the
// LDS-resident kernel where it applies; the global-memory kernel at each workgroup size and
// residency) on one colour's block sweep, then the operator workgroup size and dispatch order of
// the global solve, then its poll interval and graph replay.  Each candidate runs once to warm up and once timed.
extern "C" int ddwc_autotune(ddwc_ctx* C, double kappa, int nrhs, int prec, double* seconds_host, void* stream) {
    CK(check_common(C, kappa, nrhs, prec));
    auto t0 = std::chrono::steady_clock::now();
    const double mass = mass_of(kappa);
    double2 *b, *x;
    CK(ws_t(C, "tune_b", vec_words(C, nrhs, true), &b));
    CK(ws_t(C, "tune_x", vec_words(C, nrhs, true), &x));
    {
        Exec ex = make_exec(C, stream);
        launch_fill_hash(ex, b, vec_words(C, nrhs, true), 0x1211ULL);
    }
    auto timed = [&](auto&& run) -> double {
        double best = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            HC(hipStreamSynchronize((hipStream_t)stream));
            auto a = std::chrono::steady_clock::now();
            const int st = run();
            if (st != DDWC_OK) return -1.0;
            HC(hipStreamSynchronize((hipStream_t)stream));
            if (rep == 1) best = std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
        }
        return best;
    };
    // one schedule: the values of the options it sets
    struct Sched {
        int kernel, threads, lds;
    };
    const Sched saved = {C->opt_blk_kernel, C->opt_blk_threads, C->opt_blk_lds};
    auto set = [&](const Sched& q) {
        C->opt_blk_kernel = q.kernel;
        C->opt_blk_threads = q.threads;
        C->opt_blk_lds = q.lds;
    };
    // block solver: the LDS-resident kernel (its workgroup holds one block parity), and the
    // global-memory kernel at each workgroup size x residency (no LDS reservation, or one that
    // leaves room for 2 or 4 persistent workgroups per CU)
    int maxlds = 0;
    HC(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, C->device));
    auto per_cu = [&](int k) { return std::max(0, (maxlds / k - 2048) >> 10); };
    std::vector<Sched> cands;
    if (C->g.eo && prec != DDWC_FP64 && blk_lds_fits(C->g, C->lds_max)) cands.push_back({0, 0, 0});
    for (int T : {0, 128, 256, 512})
        for (int L : {0, per_cu(2), per_cu(4)}) cands.push_back({1, T, L});
    double best = 1e300;
    Sched pick = saved;
    for (const Sched& q : cands) {
        set(q);
        const double t = timed([&]() {
            Exec ex = make_exec(C, stream);
            BlockInfo bi;
            return block_internal(C, ex, 0, mass, b, x, nrhs, 1e-8, 5000, prec, &bi);
        });
        if (t < 0) {
            set(saved);
            return fail(DDWC_ENOCONV, "autotune: block solve failed");
        }
        if (t < best) best = t, pick = q;
    }
    set(pick);
    // global solve: operator workgroup size, then poll interval x graph replay
    auto solve_time = [&]() {
        return timed([&]() {
            Exec ex = make_exec(C, stream);
            SolveInfo si;
            return solve_internal(C, ex, mass, b, x, nrhs, 1e-8, 5000, prec, &si);
        });
    };
    const int saved_op = C->opt_op_threads, saved_order = C->opt_tile_order, saved_poll = C->opt_poll,
              saved_graphs = C->opt_graphs;
    best = 1e300;
    int po = saved_op, pr = saved_order;
    for (int nt : {128, 256, 512})
        for (int order : {0, 1}) {
            C->opt_op_threads = nt;
            C->opt_tile_order = order;
            const double t = solve_time();
            if (t < 0) {
                C->opt_op_threads = saved_op;
                C->opt_tile_order = saved_order;
                return fail(DDWC_ENOCONV, "autotune: global solve failed");
            }
            if (t < best) best = t, po = nt, pr = order;
        }
    C->opt_op_threads = po;
    C->opt_tile_order = pr;
    best = 1e300;
    int pp = saved_poll, pg = saved_graphs;
    for (int poll : {2, 4, 8})
        for (int graphs : {0, 1}) {
            C->opt_poll = poll;
            C->opt_graphs = graphs;
            const double t = solve_time();
            if (t < 0) {
                C->opt_poll = saved_poll;
                C->opt_graphs = saved_graphs;
                return fail(DDWC_ENOCONV, "autotune: global solve failed");
            }
            if (t < best) best = t, pp = poll, pg = graphs;
        }
    C->opt_poll = pp;
    C->opt_graphs = pg;
    if (seconds_host) *seconds_host = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return DDWC_OK;
}

extern "C" int ddwc_profile_enable(ddwc_ctx* C, int on) {
    CK(check_ctx(C));
    C->prof.harvest();
    C->prof.on = on != 0;
    if (on) C->prof.reset();
    return DDWC_OK;
}

extern "C" int ddwc_profile_read(ddwc_ctx* C, int kclass, long long* launches, double* total_ms, double* bytes) {
    CK(check_ctx(C));
    if (kclass < 0 || kclass >= DDWC_K_COUNT) return fail(DDWC_EINVAL, "unknown kernel class");
    C->prof.harvest();
    if (launches) *launches = C->prof.launches[kclass];
    if (total_ms) *total_ms = C->prof.ms[kclass];
    if (bytes) *bytes = C->prof.bytes[kclass];
    return DDWC_OK;
}

extern "C" int ddwc_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst) return fail(DDWC_EINVAL, "null buffer");
    if (bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
        return fail(DDWC_EINVAL, "bytes and both addresses must be multiples of 16");
    Exec ex;
    ex.stream = (hipStream_t)stream;
    ex.prof = nullptr;
    ex.nbr = nullptr;
    if (bytes) launch_stream_copy(ex, (const float4*)src, (float4*)dst, bytes / 16);
    HC(hipGetLastError());
    return DDWC_OK;
}

extern "C" const char* ddwc_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* ddwc_version(void) { return "ddwc 0.1 (gfx950)"; }
