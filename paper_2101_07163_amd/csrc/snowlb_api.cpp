// snowlb_api.cpp -- host runtime and C ABI of libsnowlb (see include/snowlb.h).
//
// Responsibilities: parameter validation (before any HIP call), device allocation of the
// structure-of-arrays population copies, the step driver (plain launches or replays of a captured
// HIP graph of K steps), the tile autotuner and its cache, FP64 diagnostics, field read-out and
// checkpoints.  Every HIP call is checked; errors are returned as status codes with a message.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/snowlb.h"
#include "snowlb_internal.h"

using namespace snowlb;

namespace {

thread_local std::string g_create_error;

const double kW9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
const double kW5[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
const int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int env_int(const char* name, int def) {
    const char* s = std::getenv(name);
    if (!s || !*s) return def;
    return std::atoi(s);
}

struct StateHeader {
    uint64_t magic;
    int32_t nx, ny, storage, flow;
    int64_t step;
    int64_t pop_bytes, phip_bytes;
    uint64_t pad[10];
};
constexpr uint64_t kMagic = 0x534e4f574c423031ull;  // "SNOWLB01"
static_assert(sizeof(StateHeader) == 128, "header size");
constexpr int64_t kHeaderBytes = 256;

}  // namespace

struct snowlb_ctx {
    snowlb_params p{};
    int device = 0;
    int esize = 4;
    DomDesc dom{};
    DomDesc* d_dom = nullptr;
    void* mem = nullptr;  // one allocation: pop[0], pop[1], phip[0], phip[1], refs[0], refs[1]
    int64_t pop_bytes = 0, phip_bytes = 0, refs_bytes = 0;
    bool local_ref = false;  // 16-bit storage: reference planes exist
    double* d_partials = nullptr;
    double* d_out = nullptr;
    double* h_out = nullptr;      // pinned, 8 doubles
    StateHeader* h_hdr = nullptr; // pinned
    hipStream_t cap_stream = nullptr;
    // tile configuration and per-configuration tile lists
    int tile = 0;
    std::vector<TileDesc*> d_tiles;
    std::vector<int> ntiles;
    // captured step loop
    hipGraphExec_t gexec = nullptr;
    int g_steps = 0, g_tile = -1;
    int par = 0;
    int64_t step = 0;
    bool inited = false;
    bool tuned = false;
    std::string err;
};

namespace {

snowlb_status fail(snowlb_ctx* c, snowlb_status s, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return s;
}

snowlb_status hip_fail(snowlb_ctx* c, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? SNOWLB_ENOMEM : SNOWLB_EDEVICE, m);
}

#define HIPCHK(c, call)                                       \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
    } while (0)

bool finite_all(const snowlb_params* p) {
    const double v[] = {p->eps, p->W0, p->tau0, p->lambda, p->L_sat, p->tau_vap, p->tau_f, p->h_drag,
                        p->kappa_N, p->rho0, p->u_in, p->U_in, p->grad_eps2, p->U0,
                        p->seed_x, p->seed_y, p->seed_r, p->init_width};
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

const char* validate_msg(const snowlb_params* p) {
    if (!p) return "params is NULL";
    if (p->nx < 2 || p->ny < 2) return "nx and ny must be >= 2";
    if (p->nx > 65536 || p->ny > 65536 || (int64_t)p->nx * p->ny > (int64_t)1 << 31)
        return "lattice too large (nx, ny <= 65536, nx*ny <= 2^31)";
    if (p->flow != 0 && p->flow != 1) return "flow must be 0 or 1";
    if (p->bc_x != SNOWLB_BC_PERIODIC && p->bc_x != SNOWLB_BC_INOUT) return "unknown bc_x";
    if (p->bc_x == SNOWLB_BC_INOUT && !p->flow) return "inflow/outflow needs flow = 1";
    if (p->storage < 0 || p->storage > 2) return "unknown storage";
    if (p->n_fold != 6 && p->n_fold != 4) return "n_fold must be 6 or 4";
    if (!finite_all(p)) return "non-finite parameter";
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
    if (p->tile < -1 || p->tile >= tile_config_count()) return "unknown tile configuration";
    return nullptr;
}

void fill_dom(snowlb_ctx* c) {
    const snowlb_params& p = c->p;
    DomDesc& d = c->dom;
    d.nx = p.nx;
    d.ny = p.ny;
    d.npop = p.flow ? 23 : 14;
    d.off_g = p.flow ? 9 : 0;
    d.off_h = d.off_g + 5;
    d.n_fold = p.n_fold;
    d.storage = p.storage;
    d.inout = p.bc_x == SNOWLB_BC_INOUT;
    const double Dphi = p.W0 * p.W0 / p.tau0;
    const double nu = (p.tau_f - 0.5) / 3.0;
    d.eps = (float)p.eps;
    d.Dphi = (float)Dphi;
    d.aniso_coef = (float)(p.kappa_N * Dphi * p.n_fold * p.eps);
    d.inv_tau0 = (float)(1.0 / p.tau0);
    d.lam = (float)p.lambda;
    d.half_Lsat = (float)(0.5 * p.L_sat);
    d.tauv_m_half = (float)(p.tau_vap - 0.5);
    d.omega_f = (float)(1.0 / p.tau_f);
    d.guo = (float)(1.0 - 0.5 / p.tau_f);
    d.kdrag = (float)(p.h_drag * nu / (4.0 * p.W0 * p.W0));
    d.grad_eps2 = p.grad_eps2;
    d.ref_f = (float)p.rho0;
    d.U_in = (float)p.U_in;
    d.u_in = (float)p.u_in;
    const double u = p.u_in;
    for (int q = 0; q < 9; ++q) {
        const double cu = kCX[q] * u;
        d.f_in[q] = (float)(kW9[q] * p.rho0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u * u));
    }
    for (int q = 0; q < 5; ++q) d.g_in[q] = (float)(kW5[q] * p.U_in * (1.0 + 3.0 * kCX[q] * u));
}

void drop_graph(snowlb_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_steps = 0;
    c->g_tile = -1;
}

snowlb_status ensure_tiles(snowlb_ctx* c, int cfg) {
    if (c->d_tiles[cfg]) return SNOWLB_OK;
    const int TX = tile_config_tx(cfg), TY = tile_config_ty(cfg);
    const int ntx = (c->p.nx + TX - 1) / TX, nty = (c->p.ny + TY - 1) / TY;
    std::vector<TileDesc> t;
    t.reserve((size_t)ntx * nty);
    for (int j = 0; j < nty; ++j)
        for (int i = 0; i < ntx; ++i) t.push_back(TileDesc{0, i * TX, j * TY, 0});
    TileDesc* d = nullptr;
    HIPCHK(c, hipMalloc(&d, t.size() * sizeof(TileDesc)));
    hipError_t e = hipMemcpy(d, t.data(), t.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(c, e, "hipMemcpy(tiles)");
    }
    c->d_tiles[cfg] = d;
    c->ntiles[cfg] = (int)t.size();
    return SNOWLB_OK;
}

snowlb_status launch_steps_plain(snowlb_ctx* c, int cfg, int n, hipStream_t s) {
    const int grid = step_grid(cfg, c->ntiles[cfg], c->p.storage, c->p.flow, c->p.bc_x);
    for (int i = 0; i < n; ++i) {
        hipError_t e = launch_step(cfg, c->p.storage, c->p.flow, c->p.bc_x, c->d_dom, c->d_tiles[cfg],
                                   c->ntiles[cfg], grid, c->par, s);
        if (e != hipSuccess) return hip_fail(c, e, "step kernel launch");
        c->par ^= 1;
        c->step += 1;
    }
    return SNOWLB_OK;
}

snowlb_status build_graph(snowlb_ctx* c, int cfg, int K) {
    drop_graph(c);
    const int grid = step_grid(cfg, c->ntiles[cfg], c->p.storage, c->p.flow, c->p.bc_x);
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int i = 0; i < K && le == hipSuccess; ++i)
        le = launch_step(cfg, c->p.storage, c->p.flow, c->p.bc_x, c->d_dom, c->d_tiles[cfg], c->ntiles[cfg],
                         grid, i & 1, c->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(c->cap_stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(c, le, "step kernel capture");
    }
    if (ee != hipSuccess) return hip_fail(c, ee, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        c->gexec = nullptr;
        return hip_fail(c, ie, "hipGraphInstantiate");
    }
    c->g_steps = K;
    c->g_tile = cfg;
    return SNOWLB_OK;
}

// Run n steps with the current tile configuration: whole graphs of K steps (K even, starting from
// copy 0) while at least K remain, single launches otherwise.
snowlb_status run_steps(snowlb_ctx* c, int n, hipStream_t s) {
    const int cfg = c->tile;
    snowlb_status st = ensure_tiles(c, cfg);
    if (st) return st;
    const int K = std::max(2, env_int("SNOWLB_GRAPH_STEPS", 32) & ~1);
    if (n < K || env_int("SNOWLB_NO_GRAPH", 0)) return launch_steps_plain(c, cfg, n, s);
    if (c->par == 1) {
        st = launch_steps_plain(c, cfg, 1, s);
        if (st) return st;
        n -= 1;
    }
    if (n >= K && (!c->gexec || c->g_tile != cfg || c->g_steps != K)) {
        st = build_graph(c, cfg, K);
        if (st) return st;
    }
    while (n >= K) {
        HIPCHK(c, hipGraphLaunch(c->gexec, s));
        c->step += K;
        n -= K;
    }
    return launch_steps_plain(c, cfg, n, s);
}

std::string tune_cache_path() {
    const char* e = std::getenv("SNOWLB_TUNE_CACHE");
    if (e && *e) return e;
    const char* h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/snowlb_tune.txt";
}

std::string tune_key(const snowlb_params& p) {
    char b[128];
    std::snprintf(b, sizeof b, "%d %d %d %d %d", p.nx, p.ny, p.storage, p.flow, p.bc_x);
    return b;
}

int tune_lookup(const snowlb_params& p) {
    FILE* f = std::fopen(tune_cache_path().c_str(), "r");
    if (!f) return -1;
    const std::string key = tune_key(p);
    char line[256];
    int found = -1;
    while (std::fgets(line, sizeof line, f)) {
        int nx, ny, st, fl, bc, cfg;
        if (std::sscanf(line, "%d %d %d %d %d %d", &nx, &ny, &st, &fl, &bc, &cfg) == 6) {
            char k[128];
            std::snprintf(k, sizeof k, "%d %d %d %d %d", nx, ny, st, fl, bc);
            if (key == k && cfg >= 0 && cfg < tile_config_count()) found = cfg;  // last entry wins
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const snowlb_params& p, int cfg) {
    const std::string path = tune_cache_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) (void)mkdir(path.substr(0, slash).c_str(), 0755);  // best effort
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", tune_key(p).c_str(), cfg);
    std::fclose(f);
}

// Time every tile configuration on a copy of the current state and keep the fastest.  The state is
// saved before and restored after, so tuning does not change the simulation.
snowlb_status autotune(snowlb_ctx* c, hipStream_t s) {
    const int64_t bytes = snowlb_state_bytes(c);
    void* save = nullptr;
    HIPCHK(c, hipMalloc(&save, (size_t)bytes));
    snowlb_status st = snowlb_save_state(c, save, bytes, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = 0;
    float best_ms = 1e30f;
    const int reps = std::max(2, env_int("SNOWLB_TUNE_STEPS", 10) & ~1);
    if (!st && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        for (int cfg = 0; cfg < tile_config_count() && !st; ++cfg) {
            st = ensure_tiles(c, cfg);
            if (st) break;
            st = launch_steps_plain(c, cfg, 2, s);
            if (st) break;
            (void)hipEventRecord(e0, s);
            st = launch_steps_plain(c, cfg, reps, s);
            (void)hipEventRecord(e1, s);
            if (st) break;
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) {
                best_ms = ms;
                best = cfg;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    snowlb_status st2 = snowlb_load_state(c, save, bytes, s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(save);
    if (st) return st;
    if (st2) return st2;
    c->tile = best;
    c->tuned = true;
    drop_graph(c);
    tune_store(c->p, best);
    return SNOWLB_OK;
}

}  // namespace

// =================================================================================================
extern "C" {

void snowlb_params_default(snowlb_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->nx = 128;
    p->ny = 128;
    p->flow = 0;
    p->bc_x = SNOWLB_BC_PERIODIC;
    p->storage = SNOWLB_STORE_FP32;
    p->n_fold = 6;
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
    p->u_in = 0.0;
    p->U_in = 0.0;
    p->grad_eps2 = 1e-10;
    p->U0 = 0.5;
    p->seed_x = 64.0;
    p->seed_y = 64.0;
    p->seed_r = 5.0;
    p->init_width = 1.0;
    p->diag_every = 0;
    p->tile = 0;
}

snowlb_status snowlb_validate(const snowlb_params* p, const char** msg_out) {
    const char* m = validate_msg(p);
    if (msg_out) *msg_out = m ? m : "";
    return m ? SNOWLB_EINVAL : SNOWLB_OK;
}

const char* snowlb_status_str(snowlb_status s) {
    switch (s) {
        case SNOWLB_OK: return "SNOWLB_OK";
        case SNOWLB_EINVAL: return "SNOWLB_EINVAL";
        case SNOWLB_ENOMEM: return "SNOWLB_ENOMEM";
        case SNOWLB_EDEVICE: return "SNOWLB_EDEVICE";
        case SNOWLB_EUNSUPPORTED: return "SNOWLB_EUNSUPPORTED";
        case SNOWLB_ENONFINITE: return "SNOWLB_ENONFINITE";
        case SNOWLB_ESTATE: return "SNOWLB_ESTATE";
    }
    return "SNOWLB_UNKNOWN";
}

const char* snowlb_last_error(const snowlb_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

snowlb_status snowlb_create(const snowlb_params* p, snowlb_ctx** out) {
    if (!out) return fail(nullptr, SNOWLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char* m = validate_msg(p)) return fail(nullptr, SNOWLB_EINVAL, m);
    snowlb_ctx* c = new (std::nothrow) snowlb_ctx();
    if (!c) return fail(nullptr, SNOWLB_ENOMEM, "host allocation failed");
    c->p = *p;
    c->esize = p->storage == SNOWLB_STORE_FP32 ? 4 : 2;
    c->d_tiles.assign(tile_config_count(), nullptr);
    c->ntiles.assign(tile_config_count(), 0);
    fill_dom(c);

    auto bail = [&](snowlb_status s) {
        g_create_error = c->err;
        snowlb_destroy(c);
        return s;
    };
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipGetDevice"));

    // geometry: rows 256-byte aligned; planes padded to 64 KiB then staggered by 9 x 256 B
    const int64_t row_align = 256 / c->esize;
    const int64_t pitch = round_up(p->nx, row_align);
    const int64_t plane_bytes =
        round_up(pitch * p->ny * c->esize, 65536) + env_int("SNOWLB_PLANE_STAGGER", 9 * 256);
    c->dom.pitch = (int32_t)pitch;
    c->dom.plane = plane_bytes / c->esize;
    c->pop_bytes = round_up(plane_bytes * c->dom.npop, 65536);
    c->phip_bytes = round_up(pitch * p->ny * 4, 65536) + env_int("SNOWLB_PLANE_STAGGER", 9 * 256);
    c->local_ref = p->storage != SNOWLB_STORE_FP32;
    int64_t rplane_bytes = 0;
    if (c->local_ref) {
        rplane_bytes = round_up(pitch * p->ny * c->esize, 65536) + env_int("SNOWLB_PLANE_STAGGER", 9 * 256);
        c->refs_bytes = round_up(rplane_bytes * (p->flow ? 4 : 1), 65536);
    }
    const int64_t total = 2 * c->pop_bytes + 2 * c->phip_bytes + 2 * c->refs_bytes;
    e = hipMalloc(&c->mem, (size_t)total);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipMalloc(state)"));
    // zero everything once: the 16-bit encodings reference phi_prev and the reference planes, which
    // must be defined even before the caller writes them
    e = hipMemset(c->mem, 0, (size_t)total);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipMemset(state)"));
    char* base = (char*)c->mem;
    c->dom.pop[0] = base;
    c->dom.pop[1] = base + c->pop_bytes;
    c->dom.phip[0] = (float*)(base + 2 * c->pop_bytes);
    c->dom.phip[1] = (float*)(base + 2 * c->pop_bytes + c->phip_bytes);
    c->dom.refs[0] = c->local_ref ? base + 2 * c->pop_bytes + 2 * c->phip_bytes : nullptr;
    c->dom.refs[1] = c->local_ref ? base + 2 * c->pop_bytes + 2 * c->phip_bytes + c->refs_bytes : nullptr;
    c->dom.rplane = rplane_bytes / c->esize;

    e = hipMalloc(&c->d_dom, sizeof(DomDesc));
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipMalloc(desc)"));
    e = hipMemcpy(c->d_dom, &c->dom, sizeof(DomDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipMemcpy(desc)"));
    e = hipMalloc(&c->d_partials, (size_t)diag_blocks(c->dom) * 8 * sizeof(double));
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipMalloc(partials)"));
    e = hipMalloc(&c->d_out, 8 * sizeof(double));
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipMalloc(out)"));
    e = hipHostMalloc(&c->h_out, 8 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipHostMalloc(out)"));
    e = hipHostMalloc(&c->h_hdr, sizeof(StateHeader), hipHostMallocDefault);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipHostMalloc(header)"));
    e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipStreamCreate"));

    c->tile = p->tile >= 0 ? p->tile : 0;
    if (p->tile == -1) {
        const int cached = tune_lookup(*p);
        if (cached >= 0) {
            c->tile = cached;
            c->tuned = true;
        }
    }
    *out = c;
    return SNOWLB_OK;
}

void snowlb_destroy(snowlb_ctx* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    drop_graph(c);
    for (TileDesc* t : c->d_tiles)
        if (t) (void)hipFree(t);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_hdr) (void)hipHostFree(c->h_hdr);
    if (c->h_out) (void)hipHostFree(c->h_out);
    if (c->d_out) (void)hipFree(c->d_out);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_dom) (void)hipFree(c->d_dom);
    if (c->mem) (void)hipFree(c->mem);
    delete c;
}

snowlb_status snowlb_init(snowlb_ctx* c, const float* U_init_dev, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    const snowlb_params& p = c->p;
    c->par = 0;
    hipError_t e = launch_init(c->dom, 0, U_init_dev, (float)p.U0, (float)p.seed_x, (float)p.seed_y,
                               (float)p.seed_r, (float)p.init_width, (float)p.u_in, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "init kernel");
    c->step = 0;
    c->inited = true;
    return SNOWLB_OK;
}

snowlb_status snowlb_step(snowlb_ctx* c, int32_t n, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (n < 0) return fail(c, SNOWLB_EINVAL, "n must be >= 0");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "step before init");
    hipStream_t s = (hipStream_t)stream;
    if (c->p.tile == -1 && !c->tuned && n > 0) {
        snowlb_status st = autotune(c, s);
        if (st) return st;
    }
    if (c->p.diag_every <= 0) return run_steps(c, n, s);
    while (n > 0) {
        const int k = std::min(n, c->p.diag_every);
        snowlb_status st = run_steps(c, k, s);
        if (st) return st;
        n -= k;
        double out[8];
        st = snowlb_diag(c, out, stream);
        if (st) return st;
    }
    return SNOWLB_OK;
}

int64_t snowlb_step_count(const snowlb_ctx* c) { return c ? c->step : -1; }

snowlb_status snowlb_read(snowlb_ctx* c, int32_t field, float* dst, int64_t elems, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (field < SNOWLB_FIELD_PHI || field > SNOWLB_FIELD_UY) return fail(c, SNOWLB_EINVAL, "unknown field");
    if (!dst || elems < (int64_t)c->p.nx * c->p.ny) return fail(c, SNOWLB_EINVAL, "dst too small");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "read before init");
    hipError_t e = launch_read(c->dom, c->par, field, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "read kernel");
    return SNOWLB_OK;
}

static int pop_q(int set) { return set == SNOWLB_POP_G ? 5 : (set == SNOWLB_POP_PHIP ? 1 : 9); }

snowlb_status snowlb_read_populations(snowlb_ctx* c, int32_t set, float* dst, int64_t elems, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (set < SNOWLB_POP_F || set > SNOWLB_POP_PHIP) return fail(c, SNOWLB_EINVAL, "unknown population set");
    if (set == SNOWLB_POP_F && !c->p.flow) return fail(c, SNOWLB_EINVAL, "no flow populations");
    if (!dst || elems < (int64_t)pop_q(set) * c->p.nx * c->p.ny) return fail(c, SNOWLB_EINVAL, "dst too small");
    hipError_t e = launch_pop_io(c->dom, c->par, set, 1, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "population read kernel");
    return SNOWLB_OK;
}

snowlb_status snowlb_write_populations(snowlb_ctx* c, int32_t set, const float* src, int64_t elems,
                                       void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (set < SNOWLB_POP_F || set > SNOWLB_POP_PHIP) return fail(c, SNOWLB_EINVAL, "unknown population set");
    if (set == SNOWLB_POP_F && !c->p.flow) return fail(c, SNOWLB_EINVAL, "no flow populations");
    if (!src || elems < (int64_t)pop_q(set) * c->p.nx * c->p.ny) return fail(c, SNOWLB_EINVAL, "src too small");
    hipError_t e = launch_pop_io(c->dom, c->par, set, 0, const_cast<float*>(src), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "population write kernel");
    c->inited = true;
    return SNOWLB_OK;
}

snowlb_status snowlb_diag(snowlb_ctx* c, double* out, void* stream) {
    if (!c || !out) return fail(c, SNOWLB_EINVAL, "NULL argument");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "diag before init");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_diag(c->dom, c->par, c->d_partials, c->d_out, s);
    if (e != hipSuccess) return hip_fail(c, e, "diag kernels");
    HIPCHK(c, hipMemcpyAsync(c->h_out, c->d_out, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    std::memcpy(out, c->h_out, 8 * sizeof(double));
    if (out[7] > 0) return fail(c, SNOWLB_ENONFINITE, "non-finite populations found");
    return SNOWLB_OK;
}

int64_t snowlb_state_bytes(const snowlb_ctx* c) {
    return c ? kHeaderBytes + c->pop_bytes + c->phip_bytes + c->refs_bytes : -1;
}

snowlb_status snowlb_save_state(snowlb_ctx* c, void* buf, int64_t bytes, void* stream) {
    if (!c || !buf) return fail(c, SNOWLB_EINVAL, "NULL argument");
    if (bytes < snowlb_state_bytes(c)) return fail(c, SNOWLB_EINVAL, "buffer too small");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "save before init");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipStreamSynchronize(s));  // the pinned header is reused by the next call
    StateHeader* h = c->h_hdr;
    std::memset(h, 0, sizeof *h);
    h->magic = kMagic;
    h->nx = c->p.nx;
    h->ny = c->p.ny;
    h->storage = c->p.storage;
    h->flow = c->p.flow;
    h->step = c->step;
    h->pop_bytes = c->pop_bytes;
    h->phip_bytes = c->phip_bytes;
    char* b = (char*)buf;
    HIPCHK(c, hipMemcpyAsync(b, h, sizeof *h, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(b + kHeaderBytes, c->dom.pop[c->par], c->pop_bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(b + kHeaderBytes + c->pop_bytes, c->dom.phip[c->par], c->phip_bytes,
                             hipMemcpyDeviceToDevice, s));
    if (c->local_ref)
        HIPCHK(c, hipMemcpyAsync(b + kHeaderBytes + c->pop_bytes + c->phip_bytes, c->dom.refs[c->par],
                                 c->refs_bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return SNOWLB_OK;
}

snowlb_status snowlb_load_state(snowlb_ctx* c, const void* buf, int64_t bytes, void* stream) {
    if (!c || !buf) return fail(c, SNOWLB_EINVAL, "NULL argument");
    if (bytes < snowlb_state_bytes(c)) return fail(c, SNOWLB_EINVAL, "buffer too small");
    hipStream_t s = (hipStream_t)stream;
    const char* b = (const char*)buf;
    HIPCHK(c, hipMemcpyAsync(c->h_hdr, b, sizeof(StateHeader), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const StateHeader* h = c->h_hdr;
    if (h->magic != kMagic || h->nx != c->p.nx || h->ny != c->p.ny || h->storage != c->p.storage ||
        h->flow != c->p.flow || h->pop_bytes != c->pop_bytes || h->phip_bytes != c->phip_bytes)
        return fail(c, SNOWLB_EINVAL, "state buffer does not match this context");
    HIPCHK(c, hipMemcpyAsync(c->dom.pop[0], b + kHeaderBytes, c->pop_bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->dom.phip[0], b + kHeaderBytes + c->pop_bytes, c->phip_bytes,
                             hipMemcpyDeviceToDevice, s));
    if (c->local_ref)
        HIPCHK(c, hipMemcpyAsync(c->dom.refs[0], b + kHeaderBytes + c->pop_bytes + c->phip_bytes,
                                 c->refs_bytes, hipMemcpyDeviceToDevice, s));
    c->par = 0;
    c->step = h->step;
    c->inited = true;
    return SNOWLB_OK;
}

int32_t snowlb_tile_count(void) { return tile_config_count(); }
const char* snowlb_tile_name(int32_t i) { return tile_config_name(i); }

snowlb_status snowlb_set_tile(snowlb_ctx* c, int32_t tile) {
    if (!c) return SNOWLB_EINVAL;
    if (tile < 0 || tile >= tile_config_count()) return fail(c, SNOWLB_EINVAL, "unknown tile configuration");
    c->tile = tile;
    c->tuned = true;
    drop_graph(c);
    return SNOWLB_OK;
}

int32_t snowlb_get_tile(const snowlb_ctx* c) { return c ? c->tile : -1; }

snowlb_status snowlb_bw_probe(void* dst, const void* src, int64_t bytes, void* stream) {
    if (!dst || !src || bytes < 0 || bytes % 16) return fail(nullptr, SNOWLB_EINVAL, "bw_probe: bad arguments");
    hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "copy kernel");
    return SNOWLB_OK;
}

}  // extern "C"
