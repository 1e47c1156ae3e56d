// snowlb3d_api.cpp -- host runtime and C ABI of the 3D step (see include/snowlb3d.h): parameter
// validation before any HIP call, one allocation per lattice (two population copies and two phi_prev
// planes in blocks of cells), graph-replayed step loops, field read-out, population exchange and
// FP64 diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "../../include/snowlb3d.h"
#include "snowlb3d_internal.h"

using namespace snowlb3d;

namespace {

thread_local std::string g_err3;  // errors of snowlb3d_create

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int env_int(const char* name, int def) {
    const char* s = std::getenv(name);
    return (s && *s) ? std::atoi(s) : def;
}

const char* validate3(const snowlb3d_params* p) {
    if (!p) return "params is NULL";
    if (p->nx < 2 || p->ny < 2 || p->nz < 2) return "nx, ny and nz must be >= 2";
    if (p->nx > 65535 || p->ny > 65535 || p->nz > 65535) return "lattice too large (nx, ny, nz <= 65535)";
    const int64_t cells = round_up(p->nx, kBX) * round_up(p->ny, kBY) * round_up(p->nz, kBZ);
    if (cells * (p->flow ? 33 : 14) * 4 > (int64_t(1) << 32))
        return "lattice too large (the populations of one copy, padded to whole blocks, within 4 GiB)";
    if (p->flow != 0 && p->flow != 1) return "flow must be 0 or 1";
    if (p->bc_x != SNOWLB_BC_PERIODIC && p->bc_x != SNOWLB_BC_INOUT) return "unknown bc_x";
    if (p->bc_x == SNOWLB_BC_INOUT && !p->flow) return "inflow/outflow needs flow = 1";
    const double v[] = {p->eps, p->W0, p->tau0, p->lambda, p->L_sat, p->tau_vap, p->tau_f, p->h_drag, p->kappa_N,
                        p->rho0, p->u_in, p->U_in, p->grad_eps2, p->U0, p->seed_x, p->seed_y, p->seed_z,
                        p->seed_r, p->init_width};
    for (double x : v)
        if (!std::isfinite(x)) return "non-finite parameter";
    if (p->eps < 0 || p->eps >= 0.5) return "eps must lie in [0, 0.5)";
    if (p->W0 <= 0 || p->tau0 <= 0) return "W0 and tau0 must be > 0";
    if (p->tau_vap <= 0.5) return "tau_vap must be > 1/2";
    if (p->flow && p->tau_f <= 0.5) return "tau_f must be > 1/2";
    if (p->flow && std::fabs(p->u_in) >= 0.1) return "|u_in| must be < 0.1 (low Mach number)";
    if (p->h_drag < 0 || p->kappa_N < 0) return "h_drag and kappa_N must be >= 0";
    if (p->flow && p->rho0 <= 0) return "rho0 must be > 0";
    if (p->grad_eps2 < 0) return "grad_eps2 must be >= 0";
    if (p->init_width <= 0) return "init_width must be > 0";
    if (p->diag_every < 0) return "diag_every must be >= 0";
    return nullptr;
}

const int kC3x[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
double w19(int q) { return q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
double w7(int q) { return q == 0 ? 0.25 : 0.125; }

}  // namespace

struct snowlb3d_ctx {
    snowlb3d_params p{};
    Dom3 dom{};
    Dom3* d_dom = nullptr;
    void* mem = nullptr;
    double* d_partials = nullptr;
    double* d_out = nullptr;
    double* h_out = nullptr;  // pinned
    hipStream_t cap = nullptr;
    hipGraphExec_t graphs[2] = {nullptr, nullptr};  // K steps, two steps (each from copy 0)
    int gsteps[2] = {0, 0};
    int par = 0;
    int64_t step = 0;
    bool inited = false;
    std::string err;
};

namespace {

snowlb_status fail3(snowlb3d_ctx* c, snowlb_status s, const std::string& m) {
    if (c) c->err = m;
    else g_err3 = m;
    return s;
}
snowlb_status hip3(snowlb3d_ctx* c, hipError_t e, const char* what) {
    return fail3(c, e == hipErrorOutOfMemory ? SNOWLB_ENOMEM : SNOWLB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK3(c, call)                                       \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip3((c), e_, #call);     \
    } while (0)

void fill_dom3(snowlb3d_ctx* c) {
    const snowlb3d_params& p = c->p;
    Dom3& d = c->dom;
    d.nx = p.nx;
    d.ny = p.ny;
    d.nz = p.nz;
    d.nbx = (p.nx + kBX - 1) / kBX;
    d.nby = (p.ny + kBY - 1) / kBY;
    d.nbz = (p.nz + kBZ - 1) / kBZ;
    d.flow = p.flow;
    d.npop = p.flow ? 33 : 14;
    d.inout = p.bc_x == SNOWLB_BC_INOUT;
    d.grad_eps2 = p.grad_eps2;
    const double Dphi = p.W0 * p.W0 / p.tau0, nu = (p.tau_f - 0.5) / 3.0;
    d.eps = (float)p.eps;
    d.Dphi = (float)Dphi;
    d.coefN = (float)(6.0 * p.kappa_N * p.eps * Dphi);
    d.inv_tau0 = (float)(1.0 / p.tau0);
    d.lam = (float)p.lambda;
    d.half_Lsat = (float)(0.5 * p.L_sat);
    d.tauv_m_half = (float)(p.tau_vap - 0.5);
    d.omega_f = (float)(1.0 / p.tau_f);
    d.guo = (float)(1.0 - 0.5 / p.tau_f);
    d.tauf_m_half = (float)(p.tau_f - 0.5);
    d.kdrag = (float)(p.h_drag * nu / (4.0 * p.W0 * p.W0));
    d.rho0 = (float)p.rho0;
    d.u_in = (float)p.u_in;
    d.U_in = (float)p.U_in;
    const double u = p.u_in;
    for (int q = 0; q < 19; ++q) {
        const double cu = kC3x[q] * u;
        d.df_in[q] = (float)(w19(q) * (p.rho0 - 1.0 + p.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * u * u)));
    }
    for (int q = 0; q < 7; ++q) d.g_in[q] = (float)(w7(q) * p.U_in * (1.0 + 4.0 * kC3x[q] * u));
}

void free3(snowlb3d_ctx* c) {
    for (hipGraphExec_t& g : c->graphs)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->h_out) (void)hipHostFree(c->h_out);
    if (c->d_out) (void)hipFree(c->d_out);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_dom) (void)hipFree(c->d_dom);
    if (c->mem) (void)hipFree(c->mem);
    c->cap = nullptr;
    c->h_out = nullptr;
    c->d_out = c->d_partials = nullptr;
    c->d_dom = nullptr;
    c->mem = nullptr;
}

snowlb_status alloc3(snowlb3d_ctx* c) {
    fill_dom3(c);
    Dom3& d = c->dom;
    const int64_t cells = (int64_t)d.nbx * d.nby * d.nbz * kBlockCells;
    const int64_t stagger = env_int("SNOWLB_BUFFER_STAGGER", 9 * 256);
    const int64_t pop_bytes = round_up(cells * d.npop * 4, 65536) + stagger;
    const int64_t phip_bytes = round_up(cells * 4, 65536) + stagger;
    const int64_t total = 2 * pop_bytes + 2 * phip_bytes;
    HIPCHK3(c, hipMalloc(&c->mem, (size_t)total));
    HIPCHK3(c, hipMemset(c->mem, 0, (size_t)total));
    char* b = (char*)c->mem;
    d.pop[0] = (float*)b;
    d.pop[1] = (float*)(b + pop_bytes);
    d.phip[0] = (float*)(b + 2 * pop_bytes);
    d.phip[1] = (float*)(b + 2 * pop_bytes + phip_bytes);
    HIPCHK3(c, hipMalloc(&c->d_dom, sizeof(Dom3)));
    HIPCHK3(c, hipMemcpy(c->d_dom, &d, sizeof(Dom3), hipMemcpyHostToDevice));
    HIPCHK3(c, hipMalloc(&c->d_partials, (size_t)diag_blocks3(d) * 9 * sizeof(double)));
    HIPCHK3(c, hipMalloc(&c->d_out, SNOWLB3D_DIAG_COUNT * sizeof(double)));
    HIPCHK3(c, hipHostMalloc(&c->h_out, SNOWLB3D_DIAG_COUNT * sizeof(double), hipHostMallocDefault));
    HIPCHK3(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    return SNOWLB_OK;
}

// Captured loop of K steps starting from copy 0, into slot `which`.
snowlb_status graph3(snowlb3d_ctx* c, int which, int K) {
    if (c->graphs[which] && c->gsteps[which] == K) return SNOWLB_OK;
    if (c->graphs[which]) (void)hipGraphExecDestroy(c->graphs[which]);
    c->graphs[which] = nullptr;
    HIPCHK3(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int i = 0; i < K && le == hipSuccess; ++i) le = launch_step3(c->dom, c->d_dom, i & 1, c->cap);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->cap, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip3(c, le, "3D step capture");
    }
    if (ee != hipSuccess) return hip3(c, ee, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return hip3(c, ie, "hipGraphInstantiate");
    c->graphs[which] = ex;
    c->gsteps[which] = K;
    return SNOWLB_OK;
}

snowlb_status plain3(snowlb3d_ctx* c, int n, hipStream_t s) {
    for (int i = 0; i < n; ++i) {
        const hipError_t e = launch_step3(c->dom, c->d_dom, c->par, s);
        if (e != hipSuccess) return hip3(c, e, "3D step launch");
        c->par ^= 1;
        c->step += 1;
    }
    return SNOWLB_OK;
}

// n steps: a single launch first if the state sits in copy 1, then K-step graphs, two-step graphs,
// and a single launch for an odd last step.
snowlb_status run3(snowlb3d_ctx* c, int n, hipStream_t s) {
    if (env_int("SNOWLB_NO_GRAPH", 0)) return plain3(c, n, s);
    const int K = std::max(2, env_int("SNOWLB_GRAPH_STEPS", 32) & ~1);
    snowlb_status st = SNOWLB_OK;
    if (c->par == 1 && n > 0) {
        if ((st = plain3(c, 1, s))) return st;
        n -= 1;
    }
    for (int which = 0; which < 2; ++which) {
        const int len = which == 0 ? K : 2;
        if (n < len) continue;
        if ((st = graph3(c, which, len))) return st;
        for (; n >= len; n -= len) {
            HIPCHK3(c, hipGraphLaunch(c->graphs[which], s));
            c->step += len;
        }
    }
    return plain3(c, n, s);
}

snowlb_status diag3(snowlb3d_ctx* c, double* out, hipStream_t s) {
    const hipError_t e = launch_diag3(c->dom, c->par, c->d_partials, c->d_out, 0.5 * c->p.L_sat, s);
    if (e != hipSuccess) return hip3(c, e, "3D diag kernels");
    HIPCHK3(c, hipMemcpyAsync(c->h_out, c->d_out, SNOWLB3D_DIAG_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK3(c, hipStreamSynchronize(s));
    std::memcpy(out, c->h_out, SNOWLB3D_DIAG_COUNT * sizeof(double));
    if (out[8] > 0) return fail3(c, SNOWLB_ENONFINITE, "non-finite populations found");
    return SNOWLB_OK;
}

int64_t cells3(const snowlb3d_ctx* c) { return (int64_t)c->p.nx * c->p.ny * c->p.nz; }

}  // namespace

extern "C" {

void snowlb3d_params_default(snowlb3d_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->nx = p->ny = p->nz = 64;
    p->bc_x = SNOWLB_BC_PERIODIC;
    p->eps = 0.05;
    p->W0 = 1.0;
    p->tau0 = 10.0;
    p->lambda = 3.0;
    p->L_sat = 1.6;
    p->tau_vap = 0.8;
    p->tau_f = 0.6;
    p->h_drag = 2.757;
    p->kappa_N = 1.0;
    p->rho0 = 1.0;
    p->grad_eps2 = 1e-10;
    p->U0 = 0.5;
    p->seed_x = p->seed_y = p->seed_z = 32.0;
    p->seed_r = 5.0;
    p->init_width = 1.0;
}

snowlb_status snowlb3d_validate(const snowlb3d_params* p, const char** msg_out) {
    const char* m = validate3(p);
    if (msg_out) *msg_out = m ? m : "";
    return m ? SNOWLB_EINVAL : SNOWLB_OK;
}

const char* snowlb3d_last_error(const snowlb3d_ctx* c) { return c ? c->err.c_str() : g_err3.c_str(); }

snowlb_status snowlb3d_create(const snowlb3d_params* p, snowlb3d_ctx** out) {
    if (!out) return fail3(nullptr, SNOWLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char* m = validate3(p)) return fail3(nullptr, SNOWLB_EINVAL, m);
    snowlb3d_ctx* c = new (std::nothrow) snowlb3d_ctx();
    if (!c) return fail3(nullptr, SNOWLB_ENOMEM, "host allocation failed");
    c->p = *p;
    const snowlb_status st = alloc3(c);
    if (st) {
        g_err3 = c->err;
        snowlb3d_destroy(c);
        return st;
    }
    *out = c;
    return SNOWLB_OK;
}

void snowlb3d_destroy(snowlb3d_ctx* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    free3(c);
    delete c;
}

snowlb_status snowlb3d_init(snowlb3d_ctx* c, const float* U_init, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    const snowlb3d_params& p = c->p;
    const hipError_t e = launch_init3(c->dom, 0, U_init, (float)p.U0, (float)p.seed_x, (float)p.seed_y,
                                      (float)p.seed_z, (float)p.seed_r, (float)p.init_width, (hipStream_t)stream);
    if (e != hipSuccess) return hip3(c, e, "3D init kernel");
    c->par = 0;
    c->step = 0;
    c->inited = true;
    return SNOWLB_OK;
}

snowlb_status snowlb3d_step(snowlb3d_ctx* c, int32_t n, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (n < 0) return fail3(c, SNOWLB_EINVAL, "n must be >= 0");
    if (!c->inited) return fail3(c, SNOWLB_ESTATE, "step before init");
    hipStream_t s = (hipStream_t)stream;
    if (c->p.diag_every <= 0) return run3(c, n, s);
    while (n > 0) {
        const int k = std::min(n, c->p.diag_every);
        snowlb_status st = run3(c, k, s);
        if (st) return st;
        n -= k;
        double out[SNOWLB3D_DIAG_COUNT];
        if ((st = diag3(c, out, s))) return st;
    }
    return SNOWLB_OK;
}

int64_t snowlb3d_step_count(const snowlb3d_ctx* c) { return c ? c->step : -1; }

snowlb_status snowlb3d_read(snowlb3d_ctx* c, int32_t field, float* dst, int64_t elems, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (field < SNOWLB3D_FIELD_PHI || field > SNOWLB3D_FIELD_UZ) return fail3(c, SNOWLB_EINVAL, "unknown field");
    if (!dst || elems < cells3(c)) return fail3(c, SNOWLB_EINVAL, "dst too small");
    if (!c->inited) return fail3(c, SNOWLB_ESTATE, "read before init");
    const hipError_t e = launch_read3(c->dom, c->par, field, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip3(c, e, "3D read kernel");
    return SNOWLB_OK;
}

static int pop_q3(int set) { return set == SNOWLB_POP_F ? 19 : (set == SNOWLB_POP_PHIP ? 1 : 7); }

snowlb_status snowlb3d_read_populations(snowlb3d_ctx* c, int32_t set, float* dst, int64_t elems, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (set < SNOWLB_POP_F || set > SNOWLB_POP_PHIP) return fail3(c, SNOWLB_EINVAL, "unknown population set");
    if (set == SNOWLB_POP_F && !c->p.flow) return fail3(c, SNOWLB_EINVAL, "no flow populations");
    if (!dst || elems < (int64_t)pop_q3(set) * cells3(c)) return fail3(c, SNOWLB_EINVAL, "dst too small");
    const hipError_t e = launch_pop_io3(c->dom, c->par, set, 1, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip3(c, e, "3D population read");
    return SNOWLB_OK;
}

snowlb_status snowlb3d_write_populations(snowlb3d_ctx* c, int32_t set, const float* src, int64_t elems,
                                         void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (set < SNOWLB_POP_F || set > SNOWLB_POP_PHIP) return fail3(c, SNOWLB_EINVAL, "unknown population set");
    if (set == SNOWLB_POP_F && !c->p.flow) return fail3(c, SNOWLB_EINVAL, "no flow populations");
    if (!src || elems < (int64_t)pop_q3(set) * cells3(c)) return fail3(c, SNOWLB_EINVAL, "src too small");
    const hipError_t e = launch_pop_io3(c->dom, c->par, set, 0, const_cast<float*>(src), (hipStream_t)stream);
    if (e != hipSuccess) return hip3(c, e, "3D population write");
    c->inited = true;
    return SNOWLB_OK;
}

snowlb_status snowlb3d_diag(snowlb3d_ctx* c, double* out, void* stream) {
    if (!c || !out) return fail3(c, SNOWLB_EINVAL, "NULL argument");
    if (!c->inited) return fail3(c, SNOWLB_ESTATE, "diag before init");
    return diag3(c, out, (hipStream_t)stream);
}

}  // extern "C"
