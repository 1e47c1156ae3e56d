// snowlb_api.cpp -- host runtime and C ABI of libsnowlb (see include/snowlb.h).
//
// Responsibilities: parameter validation (before any HIP call), device allocation of the
// structure-of-arrays population copies, the step driver shared by single contexts and batches
// (plain launches or replays of a captured HIP graph of K steps over a flat tile list), the tile /
// grid-mode autotuner and its cache, FP64 diagnostics, field read-out and checkpoints.  Every HIP
// call is checked; errors are returned as status codes with a message.
#include <hip/hip_runtime.h>
#include <sys/file.h>
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/snowlb.h"
#include "snowlb_internal.h"

using namespace snowlb;

namespace {

thread_local std::string g_free_error;  // errors of calls without a context

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
constexpr uint64_t kMagic = 0x534e4f574c423036ull;  // "SNOWLB06": 64 x 4 blocks, planes side by side, f as f - w
static_assert(sizeof(StateHeader) == 128, "header size");
constexpr int64_t kHeaderBytes = 256;

std::string hip_msg(hipError_t e, const char* what) { return std::string(what) + ": " + hipGetErrorString(e); }
snowlb_status hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? SNOWLB_ENOMEM : SNOWLB_EDEVICE; }

// ---------------------------------------------------------------------------------------------
// Step driver: a device table of domain descriptors, one flat tile list per tile configuration,
// the tile configuration and grid mode in use, the ping-pong parity and a captured graph.
// grid modes: bit 0 persistent grid; mode >> 1 the tile order (0 rows, 1 512-cell strips, 2 four strips)
constexpr int kTileOrders = 3, kLaunchModes = 2 * kTileOrders;

struct Driver {
    const DomDesc* d_doms = nullptr;  // owned by the caller
    std::vector<const DomDesc*> h_doms;  // host copies (geometry for the tile lists)
    int storage = 0, flow = 0, inout = 0, rad = 1;
    // grid_mode (launch mode): bit 0 = persistent grid (else one workgroup per tile), grid_mode >> 1 =
    // tile order; see ensure_tiles
    int tile = 0, grid_mode = 0;
    std::vector<TileDesc*> d_tiles;  // per (tile configuration, order): index list_index(cfg, mode)
    std::vector<int> ntiles;
    int par = 0;
    int64_t step = 0;
    hipStream_t cap_stream = nullptr;
    // captured step loops: [0] K steps, [1] two steps (the remainder below K), each starting from copy 0
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        int steps = 0, tile = -1, mode = -1;
    } graphs[2];
    std::string err;

    ~Driver() { release(); }

    void release() {
        drop_graph();
        for (TileDesc*& t : d_tiles)
            if (t) {
                (void)hipFree(t);
                t = nullptr;
            }
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        cap_stream = nullptr;
    }

    snowlb_status fail(snowlb_status s, const std::string& m) {
        err = m;
        return s;
    }
    snowlb_status hipfail(hipError_t e, const char* what) { return fail(hip_status(e), hip_msg(e, what)); }

    snowlb_status setup() {
        d_tiles.assign(kTileOrders * tile_config_count(), nullptr);
        ntiles.assign(kTileOrders * tile_config_count(), 0);
        hipError_t e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hipfail(e, "hipStreamCreate");
        return SNOWLB_OK;
    }

    void drop_graph() {
        for (StepGraph& g : graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            g = StepGraph{};
        }
    }

    static int list_index(int cfg, int mode) { return kTileOrders * cfg + (mode >> 1); }

    // Tile list of configuration cfg in the order of launch mode `mode`.  Row order walks each lattice
    // row of tiles by row of tiles.  The strip orders cut each lattice into vertical strips, 512 cells
    // wide (order 1) or four of nearly equal width (order 2), and walk each strip row by row: a tile
    // then shares its halo rows with tiles a strip's width away in the order instead of a lattice row
    // away, but the halo columns at a strip's edges lie in tiles that may run much later, on another
    // XCD.  Strips pay where each strip is a whole number of the XCDs' runs of the list, so that the
    // XCDs on the two sides of an edge walk it at the same time; which order wins depends on the
    // lattice (2048^2 FP16 storage: 0.1058 -> 0.0988 ms with either strip order, FP32 about even;
    // 1536^2 and 4096 x 2048: four strips 2-5 % faster; 3000^2, 6976 x 6692, 1024^2 and the
    // 64-crystal batch: strips 3-20 % slower), so the autotuner times every order.  The order does
    // not change any result.
    snowlb_status ensure_tiles(int cfg, int mode) {
        const int li = list_index(cfg, mode);
        if (d_tiles[li]) return SNOWLB_OK;
        const int TX = tile_config_tx(cfg), TY = tile_config_ty(cfg);
        std::vector<TileDesc> t;
        constexpr int kStripCells = 512;
        const int order = mode >> 1;
        for (size_t k = 0; k < h_doms.size(); ++k) {
            const DomDesc& dd = *h_doms[k];
            const int ntx = (dd.nx + TX - 1) / TX, nty = (dd.ny + TY - 1) / TY;
            const int W = order == 1 ? std::max(1, kStripCells / TX) : order == 2 ? (ntx + 3) / 4 : ntx;
            for (int s0 = 0; s0 < ntx; s0 += W)
                for (int j = 0; j < nty; ++j)
                    for (int i = s0; i < std::min(ntx, s0 + W); ++i)
                        t.push_back(TileDesc{(int32_t)k, i * TX, j * TY, 0});
        }
        if (t.size() > 0x7fffffff) return fail(SNOWLB_EINVAL, "too many tiles");
        TileDesc* d = nullptr;
        hipError_t e = hipMalloc(&d, t.size() * sizeof(TileDesc));
        if (e != hipSuccess) return hipfail(e, "hipMalloc(tiles)");
        e = hipMemcpy(d, t.data(), t.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return hipfail(e, "hipMemcpy(tiles)");
        }
        d_tiles[li] = d;
        ntiles[li] = (int)t.size();
        return SNOWLB_OK;
    }

    snowlb_status plain(int cfg, int mode, int n, hipStream_t s) {
        snowlb_status st = ensure_tiles(cfg, mode);
        if (st) return st;
        const int li = list_index(cfg, mode);
        const int grid = step_grid(cfg, ntiles[li], storage, flow, inout, rad, mode & 1);
        for (int i = 0; i < n; ++i) {
            hipError_t e = launch_step(cfg, storage, flow, inout, rad, d_doms, d_tiles[li], ntiles[li], grid, par, s);
            if (e != hipSuccess) return hipfail(e, "step kernel launch");
            par ^= 1;
            step += 1;
        }
        return SNOWLB_OK;
    }

    // Capture K steps (K even, starting from copy 0) into graph slot `which`, unless it already holds
    // them for the current tile configuration and grid mode.
    snowlb_status ensure_graph(int which, int K) {
        StepGraph& G = graphs[which];
        if (G.exec && G.steps == K && G.tile == tile && G.mode == grid_mode) return SNOWLB_OK;
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
        G = StepGraph{};
        const int li = list_index(tile, grid_mode);
        const int grid = step_grid(tile, ntiles[li], storage, flow, inout, rad, grid_mode & 1);
        hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hipfail(e, "hipStreamBeginCapture");
        hipError_t le = hipSuccess;
        for (int i = 0; i < K && le == hipSuccess; ++i)
            le = launch_step(tile, storage, flow, inout, rad, d_doms, d_tiles[li], ntiles[li], grid, i & 1,
                             cap_stream);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(cap_stream, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hipfail(le, "step kernel capture");
        }
        if (ee != hipSuccess) return hipfail(ee, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return hipfail(ie, "hipGraphInstantiate");
        G.exec = ex;
        G.steps = K;
        G.tile = tile;
        G.mode = grid_mode;
        return SNOWLB_OK;
    }

    snowlb_status replay(int which, int K, hipStream_t s) {
        hipError_t e = hipGraphLaunch(graphs[which].exec, s);
        if (e != hipSuccess) return hipfail(e, "hipGraphLaunch");
        step += K;
        return SNOWLB_OK;
    }

    // n steps with the current configuration, replayed from captured graphs: one single launch first
    // if the state sits in copy 1 (the graphs start from copy 0), then whole graphs of K steps while
    // at least K remain, then graphs of two steps, and a single launch for an odd last step.
    snowlb_status run(int n, hipStream_t s) {
        snowlb_status st = ensure_tiles(tile, grid_mode);
        if (st) return st;
        const int K = std::max(2, env_int("SNOWLB_GRAPH_STEPS", 32) & ~1);
        if (env_int("SNOWLB_NO_GRAPH", 0)) return plain(tile, grid_mode, n, s);
        if (par == 1 && n > 0) {
            st = plain(tile, grid_mode, 1, s);
            if (st) return st;
            n -= 1;
        }
        if (n >= K) {
            if ((st = ensure_graph(0, K))) return st;
            for (; n >= K; n -= K)
                if ((st = replay(0, K, s))) return st;
        }
        if (n >= 2) {
            if ((st = ensure_graph(1, 2))) return st;
            for (; n >= 2; n -= 2)
                if ((st = replay(1, 2, s))) return st;
        }
        return plain(tile, grid_mode, n, s);
    }

    // Time every (tile configuration, grid mode: launch shape and tile order) on the current state and
    // keep the fastest: all candidates first run 2 warm-up steps each (code objects loaded, tile lists
    // built), then each runs `reps` timed steps three times and its median is kept.  save / restore bracket the
    // trials, so tuning does not change the simulation.
    snowlb_status autotune(hipStream_t s, const std::function<snowlb_status()>& save,
                           const std::function<snowlb_status()>& restore) {
        snowlb_status st = save();
        if (st) return st;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            (void)restore();
            return fail(SNOWLB_EDEVICE, "hipEventCreate");
        }
        const int reps = std::max(2, env_int("SNOWLB_TUNE_STEPS", 20) & ~1);
        int best = 0, best_mode = 0;
        float best_ms = 1e30f;
        const int par0 = par;
        const int64_t step0 = step;
        for (int cfg = 0; cfg < tile_config_count() && !st; ++cfg)
            for (int mode = 0; mode < kLaunchModes && !st; ++mode) st = plain(cfg, mode, 2, s);
        for (int cfg = 0; cfg < tile_config_count() && !st; ++cfg)
            for (int mode = 0; mode < kLaunchModes && !st; ++mode) {
                float t[3];
                for (int r = 0; r < 3 && !st; ++r) {
                    (void)hipEventRecord(e0, s);
                    st = plain(cfg, mode, reps, s);
                    (void)hipEventRecord(e1, s);
                    if (st) break;
                    (void)hipEventSynchronize(e1);
                    t[r] = 0.f;
                    (void)hipEventElapsedTime(&t[r], e0, e1);
                }
                if (st) break;
                std::sort(t, t + 3);
                // a later candidate must be 1 % faster to replace the incumbent, so that near-ties
                // keep the first (simplest) configuration from run to run
                if (t[1] < 0.99f * best_ms) {
                    best_ms = t[1];
                    best = cfg;
                    best_mode = mode;
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        par = par0;
        step = step0;
        snowlb_status st2 = restore();
        if (st) return st;
        if (st2) return st2;
        tile = best;
        grid_mode = best_mode;
        drop_graph();
        return SNOWLB_OK;
    }
};

std::string tune_cache_path() {
    const char* e = std::getenv("SNOWLB_TUNE_CACHE");
    if (e && *e) return e;
    const char* h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/snowlb_tune.txt";
}

// Cache lines: "<key> <tile> <grid_mode>" where key is "<layout> nx ny storage flow bc" for one
// lattice and "<layout> batch <ndomains> <cells> storage flow bc" for a batch; <layout> names the
// memory layout the timings were taken on, so a library with another layout re-tunes.  The last
// matching line wins.
constexpr const char* kTuneLayout = "L7";
// The cache may be shared by several processes: readers take a shared lock, writers an exclusive one.
bool tune_lookup(const std::string& key, int& tile, int& mode) {
    FILE* f = std::fopen(tune_cache_path().c_str(), "r");
    if (!f) return false;
    (void)flock(fileno(f), LOCK_SH);
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        const size_t b = l.find_last_of(' ');
        if (b == std::string::npos) continue;
        const size_t a = l.find_last_of(' ', b - 1);
        if (a == std::string::npos) continue;
        if (l.substr(0, a) != key) continue;
        const int t = std::atoi(l.substr(a + 1, b - a - 1).c_str());
        const int m = std::atoi(l.substr(b + 1).c_str());
        if (t >= 0 && t < tile_config_count() && m >= 0 && m < kLaunchModes) {
            tile = t;
            mode = m;
            found = true;
        }
    }
    (void)flock(fileno(f), LOCK_UN);
    std::fclose(f);
    return found;
}

void tune_store(const std::string& key, int tile, int mode) {
    const std::string path = tune_cache_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) (void)mkdir(path.substr(0, slash).c_str(), 0755);  // best effort
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    (void)flock(fileno(f), LOCK_EX);
    std::fprintf(f, "%s %d %d\n", key.c_str(), tile, mode);
    std::fflush(f);
    (void)flock(fileno(f), LOCK_UN);
    std::fclose(f);
}

std::string tune_key(const snowlb_params& p) {
    char b[128];
    std::snprintf(b, sizeof b, "%s %d %d %d %d %d r%d", kTuneLayout, p.nx, p.ny, p.storage, p.flow, p.bc_x,
                  stencil_reach(p.stencil));
    return b;
}

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
    if (p->nx > 65536 || p->ny > 65536 ||
        round_up(p->nx, kBlockX) * round_up(p->ny, kBlockY) *
                (p->storage == SNOWLB_STORE_FP32 ? (p->flow ? 23 : 14) * 4 : (p->flow ? 27 : 15) * 2) >
            kMaxBufferBytes)
        return "lattice too large (nx, ny <= 65536, and the populations of one copy with their 16-bit "
               "references, padded to 64 x 4 blocks, within 4 GiB)";
    if (p->flow != 0 && p->flow != 1) return "flow must be 0 or 1";
    if (p->bc_x != SNOWLB_BC_PERIODIC && p->bc_x != SNOWLB_BC_INOUT) return "unknown bc_x";
    if (p->bc_x == SNOWLB_BC_INOUT && !p->flow) return "inflow/outflow needs flow = 1";
    if (p->storage < 0 || p->storage > 2) return "unknown storage";
    if (p->n_fold != 6 && p->n_fold != 4) return "n_fold must be 6 or 4";
    if (p->stencil != 2 && p->stencil != 4 && p->stencil != 6 && p->stencil != 8)
        return "stencil must be 2, 4, 6 or 8";
    if (p->symmetric != 0 && p->symmetric != 1) return "symmetric must be 0 or 1";
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

}  // namespace

// =================================================================================================
// contexts

struct snowlb_ctx {
    snowlb_params p{};
    int esize = 4;
    DomDesc dom{};
    DomDesc* d_dom = nullptr;
    void* mem = nullptr;  // one allocation: pop[0], pop[1], phip[0], phip[1], refs[0], refs[1]
    int64_t pop_bytes = 0, phip_bytes = 0;  // per copy; 16-bit references live in the population buffer
    bool local_ref = false;  // 16-bit storage: reference planes exist
    double* d_partials = nullptr;
    double* d_out = nullptr;
    double* h_out = nullptr;       // pinned, SNOWLB_DIAG_COUNT doubles
    StateHeader* h_hdr = nullptr;  // pinned
    Driver drv;
    bool inited = false;
    bool tuned = false;
    std::string err;
    // discrete adjoint: checkpoints and segment slots [pop planes | phi_prev], adjoint buffers
    struct {
        void* slots = nullptr;
        int64_t slot_bytes = 0, nslots = 0;
        int n = 0, stride = 0, nck = 0;
        bool have_forward = false;
        float* buf = nullptr;  // lambda[0], lambda[1] (15 planes each)
        double* epart = nullptr;
        double* rows = nullptr;
        double* d_out = nullptr;
        double* h_out = nullptr;  // pinned, 2 doubles
        DomDesc* d_segdoms = nullptr;  // two segment areas of (stride - 1) step descriptors each
        int nsegdoms = 0;
        // the backward pass recomputes the next interval on its own stream while the current one is
        // reversed; events order the two (index: segment area)
        hipStream_t rstream = nullptr;
        hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
        // captured segment programs (the recompute and reverse steps of one checkpoint interval),
        // each keyed by every value its kernel arguments bake in
        struct SegGraph {
            std::vector<char> key;
            hipGraphExec_t exec = nullptr;
        };
        std::vector<SegGraph> graphs;
    } adj;
};

namespace {

snowlb_status fail(snowlb_ctx* c, snowlb_status s, const std::string& msg) {
    if (c) c->err = msg;
    else g_free_error = msg;
    return s;
}

snowlb_status hip_fail(snowlb_ctx* c, hipError_t e, const char* what) {
    return fail(c, hip_status(e), hip_msg(e, what));
}

#define HIPCHK(c, call)                                         \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call);  \
    } while (0)

snowlb_status from_driver(snowlb_ctx* c, snowlb_status s) {
    if (s) c->err = c->drv.err;
    return s;
}

// eps-dependent entries of the descriptor
void fill_dom_physics_eps(snowlb_ctx* c) {
    const snowlb_params& p = c->p;
    c->dom.eps = (float)p.eps;
    c->dom.aniso_coef = (float)(p.kappa_N * (p.W0 * p.W0 / p.tau0) * p.n_fold * p.eps);
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
    d.tauf_m_half = (float)(p.tau_f - 0.5);
    d.kdrag = (float)(p.h_drag * nu / (4.0 * p.W0 * p.W0));
    d.grad_eps2 = p.grad_eps2;
    d.ref_f = (float)p.rho0;
    d.U_in = (float)p.U_in;
    d.u_in = (float)p.u_in;
    const double u = p.u_in;
    for (int q = 0; q < 9; ++q) {
        const double cu = kCX[q] * u;
        d.df_in[q] = (float)(kW9[q] * (p.rho0 - 1.0 + p.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * u * u)));
    }
    for (int q = 0; q < 5; ++q) d.g_in[q] = (float)(kW5[q] * p.U_in * (1.0 + 3.0 * kCX[q] * u));
    d.sym = p.symmetric;
    d.stencil = p.stencil;
    // gradient weights by layer |c|^2 = 1, 2, 4, 5, 8: Table 1 (E4, E6, E8) and the central difference
    static const double kGW[4][5] = {{1.0 / 2.0, 0.0, 0.0, 0.0, 0.0},
                                     {1.0 / 3.0, 1.0 / 12.0, 0.0, 0.0, 0.0},
                                     {4.0 / 15.0, 1.0 / 10.0, 1.0 / 120.0, 0.0, 0.0},
                                     {4.0 / 21.0, 4.0 / 45.0, 1.0 / 60.0, 2.0 / 315.0, 1.0 / 5040.0}};
    const int row = p.stencil / 2 - 1;
    for (int k = 0; k < 5; ++k) d.gw[k] = kGW[row][k];
}

// Allocate and describe one lattice (shared by contexts and batch members).
snowlb_status ctx_alloc(snowlb_ctx* c) {
    const snowlb_params* p = &c->p;
    c->esize = p->storage == SNOWLB_STORE_FP32 ? 4 : 2;
    fill_dom(c);
    // geometry: cells in blocks of 64 x 4 (the lattice padded up to whole blocks), each block holding
    // its planes side by side; every buffer padded to 64 KiB and then staggered by 9 x 256 B so that
    // the buffers a tile touches do not start on the same HBM channel
    const int64_t stagger = env_int("SNOWLB_BUFFER_STAGGER", 9 * 256);
    const int64_t nbx = (p->nx + kBlockX - 1) / kBlockX;
    const int64_t cells = nbx * kBlockX * round_up(p->ny, kBlockY);
    c->dom.nbx = (int32_t)nbx;
    c->dom.plane = kBlockCells;
    c->dom.rplane = kBlockCells;
    c->local_ref = p->storage != SNOWLB_STORE_FP32;
    c->dom.nqb = c->dom.npop + (c->local_ref ? (p->flow ? 4 : 1) : 0);
    c->pop_bytes = round_up(cells * c->dom.nqb * c->esize, 65536) + stagger;
    c->phip_bytes = round_up(cells * 4, 65536) + stagger;
    const int64_t total = 2 * c->pop_bytes + 2 * c->phip_bytes;
    HIPCHK(c, hipMalloc(&c->mem, (size_t)total));
    // zero everything once: the 16-bit encodings reference phi_prev and the reference planes, which
    // must be defined even before the caller writes them
    HIPCHK(c, hipMemset(c->mem, 0, (size_t)total));
    char* base = (char*)c->mem;
    c->dom.pop[0] = base;
    c->dom.pop[1] = base + c->pop_bytes;
    c->dom.phip[0] = (float*)(base + 2 * c->pop_bytes);
    c->dom.phip[1] = (float*)(base + 2 * c->pop_bytes + c->phip_bytes);
    // 16-bit references: the planes after the populations inside each block of a copy
    const int64_t rofs = (int64_t)c->dom.npop * kBlockCells * c->esize;
    c->dom.refs[0] = c->local_ref ? (char*)c->dom.pop[0] + rofs : nullptr;
    c->dom.refs[1] = c->local_ref ? (char*)c->dom.pop[1] + rofs : nullptr;
    HIPCHK(c, hipMalloc(&c->d_dom, sizeof(DomDesc)));
    HIPCHK(c, hipMemcpy(c->d_dom, &c->dom, sizeof(DomDesc), hipMemcpyHostToDevice));
    HIPCHK(c, hipMalloc(&c->d_partials, (size_t)diag_blocks(c->dom) * 8 * sizeof(double)));
    HIPCHK(c, hipMalloc(&c->d_out, SNOWLB_DIAG_COUNT * sizeof(double)));
    HIPCHK(c, hipHostMalloc(&c->h_out, SNOWLB_DIAG_COUNT * sizeof(double), hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc(&c->h_hdr, sizeof(StateHeader), hipHostMallocDefault));
    return SNOWLB_OK;
}

void adj_drop_graphs(snowlb_ctx* c) {
    for (auto& g : c->adj.graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    c->adj.graphs.clear();
}

void adj_free(snowlb_ctx* c) {
    adj_drop_graphs(c);
    if (c->adj.slots) (void)hipFree(c->adj.slots);
    if (c->adj.buf) (void)hipFree(c->adj.buf);
    if (c->adj.epart) (void)hipFree(c->adj.epart);
    if (c->adj.rows) (void)hipFree(c->adj.rows);
    if (c->adj.d_out) (void)hipFree(c->adj.d_out);
    if (c->adj.h_out) (void)hipHostFree(c->adj.h_out);
    if (c->adj.d_segdoms) (void)hipFree(c->adj.d_segdoms);
    c->adj.slots = nullptr;
    c->adj.buf = nullptr;
    c->adj.epart = c->adj.rows = c->adj.d_out = c->adj.h_out = nullptr;
    c->adj.d_segdoms = nullptr;
    for (hipEvent_t* e : {&c->adj.ev_start, &c->adj.ev_rec[0], &c->adj.ev_rec[1], &c->adj.ev_rev[0], &c->adj.ev_rev[1]})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    if (c->adj.rstream) (void)hipStreamDestroy(c->adj.rstream);
    c->adj.rstream = nullptr;
    c->adj.nslots = 0;
    c->adj.nsegdoms = 0;
    c->adj.have_forward = false;
}

void ctx_free(snowlb_ctx* c) {
    adj_free(c);
    c->drv.release();
    if (c->h_hdr) (void)hipHostFree(c->h_hdr);
    if (c->h_out) (void)hipHostFree(c->h_out);
    if (c->d_out) (void)hipFree(c->d_out);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_dom) (void)hipFree(c->d_dom);
    if (c->mem) (void)hipFree(c->mem);
    c->h_hdr = nullptr;
    c->h_out = nullptr;
    c->d_out = c->d_partials = nullptr;
    c->d_dom = nullptr;
    c->mem = nullptr;
}

snowlb_status ctx_init(snowlb_ctx* c, const float* U_init, hipStream_t s) {
    const snowlb_params& p = c->p;
    c->drv.par = 0;
    hipError_t e = launch_init(c->dom, 0, U_init, (float)p.U0, (float)p.seed_x, (float)p.seed_y, (float)p.seed_r,
                               (float)p.init_width, (float)p.u_in, s);
    if (e != hipSuccess) return hip_fail(c, e, "init kernel");
    c->drv.step = 0;
    c->inited = true;
    return SNOWLB_OK;
}

snowlb_status ctx_diag(snowlb_ctx* c, int par, double* out, hipStream_t s) {
    hipError_t e = launch_diag(c->dom, par, c->d_partials, c->d_out, 0.5 * c->p.L_sat, s);
    if (e != hipSuccess) return hip_fail(c, e, "diag kernels");
    HIPCHK(c, hipMemcpyAsync(c->h_out, c->d_out, SNOWLB_DIAG_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    std::memcpy(out, c->h_out, SNOWLB_DIAG_COUNT * sizeof(double));
    if (out[7] > 0) return fail(c, SNOWLB_ENONFINITE, "non-finite populations found");
    return SNOWLB_OK;
}

snowlb_status ctx_save(snowlb_ctx* c, int par, int64_t step, void* buf, hipStream_t s) {
    HIPCHK(c, hipStreamSynchronize(s));  // the pinned header is reused by the next call
    StateHeader* h = c->h_hdr;
    std::memset(h, 0, sizeof *h);
    h->magic = kMagic;
    h->nx = c->p.nx;
    h->ny = c->p.ny;
    h->storage = c->p.storage;
    h->flow = c->p.flow;
    h->step = step;
    h->pop_bytes = c->pop_bytes;
    h->phip_bytes = c->phip_bytes;

    char* b = (char*)buf;
    HIPCHK(c, hipMemcpyAsync(b, h, sizeof *h, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(b + kHeaderBytes, c->dom.pop[par], c->pop_bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(b + kHeaderBytes + c->pop_bytes, c->dom.phip[par], c->phip_bytes,
                             hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return SNOWLB_OK;
}

// Load a saved state into copy 0; returns its step count through *step.
snowlb_status ctx_load(snowlb_ctx* c, const void* buf, int64_t* step, hipStream_t s) {
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
    *step = h->step;
    return SNOWLB_OK;
}

int64_t ctx_state_bytes(const snowlb_ctx* c) { return kHeaderBytes + c->pop_bytes + c->phip_bytes; }

}  // namespace

// =================================================================================================
// batches

struct snowlb_batch {
    std::vector<snowlb_ctx*> doms;
    DomDesc* d_doms = nullptr;
    Driver drv;
    int64_t cells = 0;
    bool inited = false;
    bool tuned = false;
    bool autotune = false;
    std::string err;
};

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
    p->stencil = 4;
    p->symmetric = 0;
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

const char* snowlb_last_error(const snowlb_ctx* c) { return c ? c->err.c_str() : g_free_error.c_str(); }

snowlb_status snowlb_create(const snowlb_params* p, snowlb_ctx** out) {
    if (!out) return fail(nullptr, SNOWLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char* m = validate_msg(p)) return fail(nullptr, SNOWLB_EINVAL, m);
    snowlb_ctx* c = new (std::nothrow) snowlb_ctx();
    if (!c) return fail(nullptr, SNOWLB_ENOMEM, "host allocation failed");
    c->p = *p;
    snowlb_status st = ctx_alloc(c);
    if (!st) {
        c->drv.h_doms = {&c->dom};
        c->drv.d_doms = c->d_dom;
        c->drv.storage = p->storage;
        c->drv.flow = p->flow;
        c->drv.inout = p->bc_x;
        c->drv.rad = stencil_reach(p->stencil);
        st = from_driver(c, c->drv.setup());
    }
    if (st) {
        g_free_error = c->err;
        snowlb_destroy(c);
        return st;
    }
    c->drv.tile = p->tile >= 0 ? p->tile : 0;
    if (p->tile == -1 && tune_lookup(tune_key(*p), c->drv.tile, c->drv.grid_mode)) c->tuned = true;
    *out = c;
    return SNOWLB_OK;
}

void snowlb_destroy(snowlb_ctx* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    ctx_free(c);
    delete c;
}

snowlb_status snowlb_init(snowlb_ctx* c, const float* U_init_dev, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    return ctx_init(c, U_init_dev, (hipStream_t)stream);
}

snowlb_status snowlb_step(snowlb_ctx* c, int32_t n, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (n < 0) return fail(c, SNOWLB_EINVAL, "n must be >= 0");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "step before init");
    hipStream_t s = (hipStream_t)stream;
    if (c->p.tile == -1 && !c->tuned && n > 0) {
        void* save = nullptr;
        const int64_t bytes = ctx_state_bytes(c);
        HIPCHK(c, hipMalloc(&save, (size_t)bytes));
        const int par0 = c->drv.par;
        const int64_t step0 = c->drv.step;
        snowlb_status st = c->drv.autotune(
            s, [&] { return ctx_save(c, par0, step0, save, s); },
            [&] {
                int64_t st_step = 0;
                snowlb_status r = ctx_load(c, save, &st_step, s);
                (void)hipStreamSynchronize(s);
                c->drv.par = 0;
                c->drv.step = st_step;
                return r;
            });
        (void)hipFree(save);
        if (st) return from_driver(c, st);
        c->tuned = true;
        tune_store(tune_key(c->p), c->drv.tile, c->drv.grid_mode);
    }
    if (c->p.diag_every <= 0) return from_driver(c, c->drv.run(n, s));
    while (n > 0) {
        const int k = std::min(n, c->p.diag_every);
        snowlb_status st = from_driver(c, c->drv.run(k, s));
        if (st) return st;
        n -= k;
        double out[SNOWLB_DIAG_COUNT];
        st = ctx_diag(c, c->drv.par, out, s);
        if (st) return st;
    }
    return SNOWLB_OK;
}

int64_t snowlb_step_count(const snowlb_ctx* c) { return c ? c->drv.step : -1; }

snowlb_status snowlb_read(snowlb_ctx* c, int32_t field, float* dst, int64_t elems, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (field < SNOWLB_FIELD_PHI || field > SNOWLB_FIELD_UY) return fail(c, SNOWLB_EINVAL, "unknown field");
    if (!dst || elems < (int64_t)c->p.nx * c->p.ny) return fail(c, SNOWLB_EINVAL, "dst too small");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "read before init");
    hipError_t e = launch_read(c->dom, c->drv.par, field, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "read kernel");
    return SNOWLB_OK;
}

static int pop_q(int set) { return set == SNOWLB_POP_G ? 5 : (set == SNOWLB_POP_PHIP ? 1 : 9); }

snowlb_status snowlb_read_populations(snowlb_ctx* c, int32_t set, float* dst, int64_t elems, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (set < SNOWLB_POP_F || set > SNOWLB_POP_PHIP) return fail(c, SNOWLB_EINVAL, "unknown population set");
    if (set == SNOWLB_POP_F && !c->p.flow) return fail(c, SNOWLB_EINVAL, "no flow populations");
    if (!dst || elems < (int64_t)pop_q(set) * c->p.nx * c->p.ny) return fail(c, SNOWLB_EINVAL, "dst too small");
    hipError_t e = launch_pop_io(c->dom, c->drv.par, set, 1, dst, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "population read kernel");
    return SNOWLB_OK;
}

snowlb_status snowlb_write_field(snowlb_ctx* c, int32_t field, const float* src, int64_t elems, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (field != SNOWLB_FIELD_PHI && field != SNOWLB_FIELD_U)
        return fail(c, SNOWLB_EINVAL, "only SNOWLB_FIELD_PHI and SNOWLB_FIELD_U can be written");
    if (!src || elems < (int64_t)c->p.nx * c->p.ny) return fail(c, SNOWLB_EINVAL, "src too small");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "write_field before init");
    hipError_t e = launch_write_field(c->dom, c->drv.par, field, src, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "field write kernel");
    return SNOWLB_OK;
}

snowlb_status snowlb_write_populations(snowlb_ctx* c, int32_t set, const float* src, int64_t elems,
                                       void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (set < SNOWLB_POP_F || set > SNOWLB_POP_PHIP) return fail(c, SNOWLB_EINVAL, "unknown population set");
    if (set == SNOWLB_POP_F && !c->p.flow) return fail(c, SNOWLB_EINVAL, "no flow populations");
    if (!src || elems < (int64_t)pop_q(set) * c->p.nx * c->p.ny) return fail(c, SNOWLB_EINVAL, "src too small");
    hipError_t e = launch_pop_io(c->dom, c->drv.par, set, 0, const_cast<float*>(src), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "population write kernel");
    c->inited = true;
    return SNOWLB_OK;
}

snowlb_status snowlb_diag(snowlb_ctx* c, double* out, void* stream) {
    if (!c || !out) return fail(c, SNOWLB_EINVAL, "NULL argument");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "diag before init");
    return ctx_diag(c, c->drv.par, out, (hipStream_t)stream);
}

snowlb_status snowlb_diag_noalloc(snowlb_ctx* c, double* out_dev, void* stream) {
    if (!c || !out_dev) return fail(c, SNOWLB_EINVAL, "NULL argument");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "diag before init");
    if (diag_blocks(c->dom) > kDiagMaxBlocks)
        return fail(c, SNOWLB_EINVAL, "diagnostics need more partials than the static scratch holds");
    double* scr = nullptr;  // this device's copy of the static scratch array
    hipError_t e = diag_scratch(&scr);
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    e = launch_diag(c->dom, c->drv.par, scr, out_dev, 0.5 * c->p.L_sat, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "diag kernels");
    return SNOWLB_OK;
}

int64_t snowlb_state_bytes(const snowlb_ctx* c) { return c ? ctx_state_bytes(c) : -1; }

snowlb_status snowlb_save_state(snowlb_ctx* c, void* buf, int64_t bytes, void* stream) {
    if (!c || !buf) return fail(c, SNOWLB_EINVAL, "NULL argument");
    if (bytes < ctx_state_bytes(c)) return fail(c, SNOWLB_EINVAL, "buffer too small");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "save before init");
    return ctx_save(c, c->drv.par, c->drv.step, buf, (hipStream_t)stream);
}

snowlb_status snowlb_load_state(snowlb_ctx* c, const void* buf, int64_t bytes, void* stream) {
    if (!c || !buf) return fail(c, SNOWLB_EINVAL, "NULL argument");
    if (bytes < ctx_state_bytes(c)) return fail(c, SNOWLB_EINVAL, "buffer too small");
    int64_t step = 0;
    snowlb_status st = ctx_load(c, buf, &step, (hipStream_t)stream);
    if (st) return st;
    c->drv.par = 0;
    c->drv.step = step;
    c->inited = true;
    return SNOWLB_OK;
}

int32_t snowlb_tile_count(void) { return tile_config_count(); }
const char* snowlb_tile_name(int32_t i) { return tile_config_name(i); }

snowlb_status snowlb_set_tile(snowlb_ctx* c, int32_t tile) {
    if (!c) return SNOWLB_EINVAL;
    if (tile < 0 || tile >= tile_config_count()) return fail(c, SNOWLB_EINVAL, "unknown tile configuration");
    c->drv.tile = tile;
    c->tuned = true;
    c->drv.drop_graph();
    return SNOWLB_OK;
}

int32_t snowlb_get_tile(const snowlb_ctx* c) { return c ? c->drv.tile : -1; }

snowlb_status snowlb_set_grid_mode(snowlb_ctx* c, int32_t mode) {
    if (!c) return SNOWLB_EINVAL;
    if (mode < 0 || mode >= kLaunchModes) return fail(c, SNOWLB_EINVAL, "grid mode must be 0..5");
    c->drv.grid_mode = mode;
    c->tuned = true;
    c->drv.drop_graph();
    return SNOWLB_OK;
}

int32_t snowlb_get_grid_mode(const snowlb_ctx* c) { return c ? c->drv.grid_mode : -1; }

snowlb_status snowlb_set_eps(snowlb_ctx* c, double eps) {
    if (!c) return SNOWLB_EINVAL;
    if (!std::isfinite(eps) || eps < 0 || eps >= 0.5) return fail(c, SNOWLB_EINVAL, "eps must lie in [0, 0.5)");
    c->p.eps = eps;
    fill_dom_physics_eps(c);
    // steps already queued on any stream read the descriptor: let them finish with the old value
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(c->d_dom, &c->dom, sizeof(DomDesc), hipMemcpyHostToDevice));
    return SNOWLB_OK;
}

// ---------------------------------------------------------------------------------------------- adjoint

static snowlb_status adj_check(snowlb_ctx* c) {
    if (c->p.flow || c->p.bc_x != SNOWLB_BC_PERIODIC || c->p.storage != SNOWLB_STORE_FP32 || c->p.stencil != 4 ||
        c->p.symmetric)
        return fail(c, SNOWLB_EUNSUPPORTED,
                    "the adjoint supports flow = 0, periodic x, FP32 storage, the E4 gradient and the one-sided "
                    "diffusivity");
    return SNOWLB_OK;
}

static char* adj_slot(snowlb_ctx* c, int64_t k) { return (char*)c->adj.slots + k * c->adj.slot_bytes; }
// cells of the lattice padded to whole 64 x 4 blocks (the size of one plane of the cell order)
static int64_t adj_cells(const snowlb_ctx* c) { return (int64_t)c->dom.nbx * kBlockX * round_up(c->p.ny, kBlockY); }

snowlb_status snowlb_adj_forward(snowlb_ctx* c, int32_t n, int32_t stride, void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (snowlb_status st = adj_check(c)) return st;
    if (n < 1 || stride < 0) return fail(c, SNOWLB_EINVAL, "need n >= 1 and stride >= 0");
    if (!c->inited) return fail(c, SNOWLB_ESTATE, "adjoint forward before init");
    hipStream_t s = (hipStream_t)stream;
    const int st = stride > 0 ? stride : (int)std::ceil(std::sqrt((double)n));
    const int nck = (n + st - 1) / st;
    const int64_t slot_bytes = c->pop_bytes + c->phip_bytes;
    const int64_t need = (int64_t)nck + 2 * (int64_t)st;  // checkpoints, then two segment areas
    if (c->adj.nslots < need || c->adj.slot_bytes != slot_bytes) {
        if (c->adj.slots) (void)hipFree(c->adj.slots);
        c->adj.slots = nullptr;
        c->adj.nslots = 0;
        HIPCHK(c, hipMalloc(&c->adj.slots, (size_t)(need * slot_bytes)));
        c->adj.nslots = need;
        c->adj.slot_bytes = slot_bytes;
        c->adj.nsegdoms = 0;  // segment descriptors point into the slots
    }
    c->adj.n = n;
    c->adj.stride = st;
    c->adj.nck = nck;
    for (int k = 0; k < nck; ++k) {
        char* sl = adj_slot(c, k);
        HIPCHK(c, hipMemcpyAsync(sl, c->dom.pop[c->drv.par], c->pop_bytes, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(sl + c->pop_bytes, c->dom.phip[c->drv.par], c->phip_bytes, hipMemcpyDeviceToDevice, s));
        const int len = std::min(st, n - k * st);
        snowlb_status r = from_driver(c, c->drv.run(len, s));
        if (r) return r;
    }
    c->adj.have_forward = true;
    return SNOWLB_OK;
}

// First slot of segment area a (two areas of `stride` states follow the checkpoints).
static int64_t adj_area_slot(const snowlb_ctx* c, int a) { return (int64_t)c->adj.nck + (int64_t)a * c->adj.stride; }

// Captured programs of one checkpoint interval of length len in segment area `area`: kind 0, the
// (len - 1) recompute steps from the checkpoint copied into the area's first slot; kind 1, the len
// reverse steps over the area's states, starting from lambda[cur].  Programs are cached on the
// context, keyed by every value their kernel arguments bake in.
static snowlb_status adj_graph(snowlb_ctx* c, int kind, AdjDesc A, float* const lam[2], int area, int len, int cur,
                               int grid, hipGraphExec_t* out) {
    Driver& D = c->drv;
    struct Key {
        AdjDesc A;
        const void* lam0;
        const void* lam1;
        const void* slots;
        const void* segdoms;
        const void* tiles;
        int64_t slot_bytes;
        int32_t nck, stride, tile, grid, storage, len, cur, kind, area, pad;
    } key;
    std::memset(&key, 0, sizeof key);
    if (kind == 1) {
        key.A = A;
        key.A.st = key.A.lin = key.A.lppin = nullptr;
        key.A.lout = key.A.lppout = nullptr;
        key.lam0 = lam[0];
        key.lam1 = lam[1];
        key.cur = cur;
    } else {
        key.segdoms = c->adj.d_segdoms;
        key.tiles = D.d_tiles[Driver::list_index(D.tile, D.grid_mode)];
        key.tile = D.tile;
        key.grid = grid;
        key.storage = c->p.storage;
    }
    key.slots = c->adj.slots;
    key.slot_bytes = c->adj.slot_bytes;
    key.nck = c->adj.nck;
    key.stride = c->adj.stride;
    key.len = len;
    key.kind = kind;
    key.area = area;
    const char* kb = reinterpret_cast<const char*>(&key);
    for (auto& sg : c->adj.graphs)
        if (sg.key.size() == sizeof key && std::memcmp(sg.key.data(), kb, sizeof key) == 0) {
            *out = sg.exec;
            return SNOWLB_OK;
        }
    hipStream_t cs = D.cap_stream;
    HIPCHK(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    if (kind == 0) {
        const DomDesc* sd = c->adj.d_segdoms + (int64_t)area * std::max(c->adj.stride - 1, 1);
        for (int i = 0; i + 1 < len && le == hipSuccess; ++i)
            le = launch_step(D.tile, c->p.storage, 0, 0, 1, sd + i, D.d_tiles[Driver::list_index(D.tile, D.grid_mode)],
                             D.ntiles[Driver::list_index(D.tile, D.grid_mode)], grid, 0, cs);
    } else {
        const int64_t base = adj_area_slot(c, area);
        for (int i = len - 1; i >= 0 && le == hipSuccess; --i) {
            A.st = (const float*)adj_slot(c, base + i);
            A.lin = lam[cur];
            A.lout = lam[1 - cur];
            A.lppin = lam[cur] + kAdjPlanes * adj_cells(c);
            A.lppout = lam[1 - cur] + kAdjPlanes * adj_cells(c);
            le = launch_adj_step(A, cs);
            cur ^= 1;
        }
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(c, le, "adjoint segment capture");
    }
    if (ee != hipSuccess) return hip_fail(c, ee, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return hip_fail(c, ie, "hipGraphInstantiate");
    c->adj.graphs.push_back({std::vector<char>(kb, kb + sizeof key), ex});
    *out = ex;
    return SNOWLB_OK;
}

snowlb_status snowlb_adj_backward(snowlb_ctx* c, const float* dphi, float* dU, double* deps, double* dU0,
                                  void* stream) {
    if (!c) return SNOWLB_EINVAL;
    if (snowlb_status st = adj_check(c)) return st;
    if (!dphi || !dU || !deps || !dU0) return fail(c, SNOWLB_EINVAL, "NULL argument");
    if (!c->adj.have_forward) return fail(c, SNOWLB_ESTATE, "adjoint backward before adjoint forward");
    hipStream_t s = (hipStream_t)stream;
    // One backward pass uses at most 12 programs (recompute: 2 areas x 2 interval lengths; reverse: 2
    // areas x 2 lambda parities x 2 lengths).  Programs are only dropped here, while none can be in
    // flight: the previous pass synchronised its stream before returning.
    if (c->adj.graphs.size() > 4) adj_drop_graphs(c);
    // lambda buffers: the 14 planes of g and h in the populations' cell order, then phi_prev's plane
    const int64_t cells = adj_cells(c);
    AdjDesc A{};
    A.nx = c->p.nx;
    A.ny = c->p.ny;
    A.nbx = c->dom.nbx;
    A.n_fold = c->p.n_fold;
    A.grad_eps2 = c->p.grad_eps2;
    A.eps = c->dom.eps;
    A.Dphi = c->dom.Dphi;
    A.coefN = (float)(c->p.kappa_N * (c->p.W0 * c->p.W0 / c->p.tau0) * c->p.n_fold);
    A.inv_tau0 = c->dom.inv_tau0;
    A.lam = c->dom.lam;
    A.half_Lsat = c->dom.half_Lsat;
    A.tauv_m_half = c->dom.tauv_m_half;
    const int nblk = adj_blocks(A);
    if (!c->adj.buf) {
        HIPCHK(c, hipMalloc(&c->adj.buf, (size_t)(2 * (kAdjPlanes + 1) * cells * 4)));
        HIPCHK(c, hipMalloc(&c->adj.epart, (size_t)nblk * sizeof(double)));
        HIPCHK(c, hipMalloc(&c->adj.rows, (size_t)c->p.ny * sizeof(double)));
        HIPCHK(c, hipMalloc(&c->adj.d_out, 2 * sizeof(double)));
        HIPCHK(c, hipHostMalloc(&c->adj.h_out, 2 * sizeof(double), hipHostMallocDefault));
    }
    const int st = c->adj.stride, n = c->adj.n;
    const int per_area = std::max(st - 1, 1);
    {
        // Step i of a recompute in area `ar` reads slot i of the area and writes slot i + 1.  The
        // descriptors are rebuilt on every call from the context's current domain (eps may have
        // changed since the forward pass through snowlb_set_eps) and the current slot layout (the
        // segment areas follow the checkpoints, so they move when the checkpoint count changes).
        std::vector<DomDesc> h((size_t)(2 * per_area), c->dom);
        for (int ar = 0; ar < 2; ++ar)
            for (int i = 0; i + 1 < st; ++i) {
                DomDesc& d = h[(size_t)(ar * per_area + i)];
                char* a = adj_slot(c, adj_area_slot(c, ar) + i);
                char* b = adj_slot(c, adj_area_slot(c, ar) + i + 1);
                d.pop[0] = a;
                d.pop[1] = b;
                d.phip[0] = (float*)(a + c->pop_bytes);
                d.phip[1] = (float*)(b + c->pop_bytes);
            }
        if (c->adj.nsegdoms < (int)h.size()) {
            if (c->adj.d_segdoms) (void)hipFree(c->adj.d_segdoms);
            c->adj.d_segdoms = nullptr;
            c->adj.nsegdoms = 0;
            HIPCHK(c, hipMalloc(&c->adj.d_segdoms, h.size() * sizeof(DomDesc)));
            c->adj.nsegdoms = (int)h.size();
        }
        // the previous backward pass returned only after all of its work (both streams) was done,
        // so once the caller's stream has drained nothing reads the descriptors any more
        HIPCHK(c, hipStreamSynchronize(s));
        HIPCHK(c, hipMemcpy(c->adj.d_segdoms, h.data(), h.size() * sizeof(DomDesc), hipMemcpyHostToDevice));
    }
    float* lam[2] = {c->adj.buf, c->adj.buf + (kAdjPlanes + 1) * cells};
    A.epart = c->adj.epart;
    HIPCHK(c, hipMemsetAsync(c->adj.epart, 0, (size_t)nblk * sizeof(double), s));
    A.lout = lam[0];
    A.lppout = lam[0] + kAdjPlanes * cells;
    hipError_t e = launch_adj_seed(A, dphi, s);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint seed kernel");
    Driver& D = c->drv;
    snowlb_status r = from_driver(c, D.ensure_tiles(D.tile, D.grid_mode));
    if (r) return r;
    const int grid = step_grid(D.tile, D.ntiles[Driver::list_index(D.tile, D.grid_mode)], c->p.storage, 0, 0, 1,
                               D.grid_mode & 1);
    // Checkpoint intervals are reversed from the last to the first.  Interval k lives in segment area
    // k % 2: its checkpoint is copied into the area's first slot, (len - 1) recompute steps fill the
    // rest, and len reverse steps consume it.  With overlap (the default), interval k - 1 is
    // recomputed on the context's second stream while interval k is reversed on the caller's: the
    // recompute waits for the reverse of interval k + 1 (the last user of its area), and each reverse
    // waits for its own recompute.  Every kernel sees the same inputs as in the serial order, so the
    // results are bitwise the same.
    const bool overlap = env_int("SNOWLB_ADJ_OVERLAP", 1) != 0;
    if (overlap && !c->adj.rstream) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->adj.rstream, hipStreamNonBlocking));
        for (hipEvent_t* ev : {&c->adj.ev_start, &c->adj.ev_rec[0], &c->adj.ev_rec[1], &c->adj.ev_rev[0],
                               &c->adj.ev_rev[1]})
            HIPCHK(c, hipEventCreateWithFlags(ev, hipEventDisableTiming));
    }
    hipStream_t rs = overlap ? c->adj.rstream : s;
    auto recompute = [&](int k) -> snowlb_status {
        const int len = std::min(st, n - k * st), ar = k & 1;
        HIPCHK(c, hipMemcpyAsync(adj_slot(c, adj_area_slot(c, ar)), adj_slot(c, k), (size_t)c->adj.slot_bytes,
                                 hipMemcpyDeviceToDevice, rs));
        if (len > 1) {
            hipGraphExec_t g = nullptr;
            if (snowlb_status r2 = adj_graph(c, 0, A, lam, ar, len, 0, grid, &g)) return r2;
            HIPCHK(c, hipGraphLaunch(g, rs));
        }
        if (overlap) HIPCHK(c, hipEventRecord(c->adj.ev_rec[ar], rs));
        return SNOWLB_OK;
    };
    if (overlap) {  // the second stream starts after everything queued on the caller's stream so far
        HIPCHK(c, hipEventRecord(c->adj.ev_start, s));
        HIPCHK(c, hipStreamWaitEvent(rs, c->adj.ev_start, 0));
    }
    if (snowlb_status r2 = recompute(c->adj.nck - 1)) return r2;
    int cur = 0;
    for (int k = c->adj.nck - 1; k >= 0; --k) {
        const int len = std::min(st, n - k * st), ar = k & 1;
        if (overlap) HIPCHK(c, hipStreamWaitEvent(s, c->adj.ev_rec[ar], 0));
        hipGraphExec_t g = nullptr;
        if (snowlb_status r2 = adj_graph(c, 1, A, lam, ar, len, cur, grid, &g)) return r2;
        HIPCHK(c, hipGraphLaunch(g, s));
        cur ^= len & 1;
        if (overlap) HIPCHK(c, hipEventRecord(c->adj.ev_rev[ar], s));
        if (k > 0) {
            // interval k - 1 uses area (k - 1) % 2, last read by the reverse of interval k + 1
            if (overlap && k + 1 < c->adj.nck) HIPCHK(c, hipStreamWaitEvent(rs, c->adj.ev_rev[(k + 1) & 1], 0));
            if (snowlb_status r2 = recompute(k - 1)) return r2;
        }
    }
    A.lin = lam[cur];
    e = launch_adj_finish(A, dU, c->adj.rows, c->adj.d_out, s);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint reduction kernels");
    HIPCHK(c, hipMemcpyAsync(c->adj.h_out, c->adj.d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    *deps = c->adj.h_out[0];
    *dU0 = c->adj.h_out[1];
    return SNOWLB_OK;
}

// ---------------------------------------------------------------------------------------------- batch

const char* snowlb_batch_last_error(const snowlb_batch* b) { return b ? b->err.c_str() : g_free_error.c_str(); }

void snowlb_batch_destroy(snowlb_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    b->drv.release();
    if (b->d_doms) (void)hipFree(b->d_doms);
    for (snowlb_ctx* c : b->doms) snowlb_destroy(c);
    delete b;
}

snowlb_status snowlb_batch_create(const snowlb_params* params, int32_t n, snowlb_batch** out) {
    if (!out) return fail(nullptr, SNOWLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || n < 1) return fail(nullptr, SNOWLB_EINVAL, "need params and n >= 1");
    for (int i = 0; i < n; ++i) {
        if (const char* m = validate_msg(&params[i]))
            return fail(nullptr, SNOWLB_EINVAL, "domain " + std::to_string(i) + ": " + m);
        const snowlb_params& a = params[0];
        const snowlb_params& p = params[i];
        if (p.flow != a.flow || p.bc_x != a.bc_x || p.storage != a.storage || p.n_fold != a.n_fold ||
            stencil_reach(p.stencil) != stencil_reach(a.stencil))
            return fail(nullptr, SNOWLB_EINVAL,
                        "batch domains must share flow, bc_x, storage, n_fold and the stencil reach (E2/E4 or E6/E8)");
    }
    snowlb_batch* b = new (std::nothrow) snowlb_batch();
    if (!b) return fail(nullptr, SNOWLB_ENOMEM, "host allocation failed");
    auto bail = [&](snowlb_status s, const std::string& m) {
        g_free_error = m;
        snowlb_batch_destroy(b);
        return s;
    };
    std::vector<DomDesc> h;
    for (int i = 0; i < n; ++i) {
        snowlb_ctx* c = nullptr;
        snowlb_params p = params[i];
        p.tile = 0;
        snowlb_status st = snowlb_create(&p, &c);
        if (st) return bail(st, "domain " + std::to_string(i) + ": " + g_free_error);
        b->doms.push_back(c);
        h.push_back(c->dom);
        b->cells += (int64_t)p.nx * p.ny;
    }
    hipError_t e = hipMalloc(&b->d_doms, h.size() * sizeof(DomDesc));
    if (e != hipSuccess) return bail(hip_status(e), hip_msg(e, "hipMalloc(domains)"));
    e = hipMemcpy(b->d_doms, h.data(), h.size() * sizeof(DomDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_status(e), hip_msg(e, "hipMemcpy(domains)"));
    for (snowlb_ctx* c : b->doms) b->drv.h_doms.push_back(&c->dom);
    b->drv.d_doms = b->d_doms;
    b->drv.storage = params[0].storage;
    b->drv.flow = params[0].flow;
    b->drv.inout = params[0].bc_x;
    b->drv.rad = stencil_reach(params[0].stencil);
    snowlb_status st = b->drv.setup();
    if (st) return bail(st, b->drv.err);
    b->drv.tile = params[0].tile >= 0 ? params[0].tile : 0;
    b->autotune = params[0].tile == -1;
    *out = b;
    return SNOWLB_OK;
}

int32_t snowlb_batch_size(const snowlb_batch* b) { return b ? (int32_t)b->doms.size() : -1; }
int64_t snowlb_batch_cells(const snowlb_batch* b) { return b ? b->cells : -1; }
int64_t snowlb_batch_step_count(const snowlb_batch* b) { return b ? b->drv.step : -1; }

snowlb_status snowlb_batch_init(snowlb_batch* b, void* stream) {
    if (!b) return SNOWLB_EINVAL;
    for (snowlb_ctx* c : b->doms) {
        snowlb_status st = ctx_init(c, nullptr, (hipStream_t)stream);
        if (st) {
            b->err = c->err;
            return st;
        }
    }
    b->drv.par = 0;
    b->drv.step = 0;
    b->inited = true;
    return SNOWLB_OK;
}

static std::string batch_key(const snowlb_batch* b) {
    const snowlb_params& p = b->doms[0]->p;
    char k[160];
    std::snprintf(k, sizeof k, "%s batch %d %lld %d %d %d r%d", kTuneLayout, (int)b->doms.size(), (long long)b->cells,
                  p.storage, p.flow, p.bc_x, stencil_reach(p.stencil));
    return k;
}

snowlb_status snowlb_batch_step(snowlb_batch* b, int32_t n, void* stream) {
    if (!b) return SNOWLB_EINVAL;
    if (n < 0) {
        b->err = "n must be >= 0";
        return SNOWLB_EINVAL;
    }
    if (!b->inited) {
        b->err = "step before init";
        return SNOWLB_ESTATE;
    }
    hipStream_t s = (hipStream_t)stream;
    if (b->autotune && !b->tuned && n > 0) {
        if (tune_lookup(batch_key(b), b->drv.tile, b->drv.grid_mode)) {
            b->tuned = true;
        } else {
            std::vector<void*> saves(b->doms.size(), nullptr);
            snowlb_status st = SNOWLB_OK;
            for (size_t i = 0; i < b->doms.size() && !st; ++i) {
                hipError_t e = hipMalloc(&saves[i], (size_t)ctx_state_bytes(b->doms[i]));
                if (e != hipSuccess) {
                    st = hip_status(e);
                    b->err = hip_msg(e, "hipMalloc(tune save)");
                }
            }
            const int par0 = b->drv.par;
            const int64_t step0 = b->drv.step;
            if (!st)
                st = b->drv.autotune(
                    s,
                    [&] {
                        for (size_t i = 0; i < b->doms.size(); ++i) {
                            snowlb_status r = ctx_save(b->doms[i], par0, step0, saves[i], s);
                            if (r) return r;
                        }
                        return SNOWLB_OK;
                    },
                    [&] {
                        int64_t stp = 0;
                        for (size_t i = 0; i < b->doms.size(); ++i) {
                            snowlb_status r = ctx_load(b->doms[i], saves[i], &stp, s);
                            if (r) return r;
                        }
                        (void)hipStreamSynchronize(s);
                        b->drv.par = 0;
                        b->drv.step = step0;
                        return SNOWLB_OK;
                    });
            for (void* p : saves)
                if (p) (void)hipFree(p);
            if (st) {
                if (b->err.empty()) b->err = b->drv.err;
                return st;
            }
            b->tuned = true;
            tune_store(batch_key(b), b->drv.tile, b->drv.grid_mode);
        }
    }
    snowlb_status st = b->drv.run(n, s);
    if (st) b->err = b->drv.err;
    return st;
}

snowlb_status snowlb_batch_read(snowlb_batch* b, int32_t i, int32_t field, float* dst, int64_t elems, void* stream) {
    if (!b || i < 0 || i >= (int32_t)b->doms.size()) return SNOWLB_EINVAL;
    snowlb_ctx* c = b->doms[i];
    c->drv.par = b->drv.par;
    c->drv.step = b->drv.step;
    snowlb_status st = snowlb_read(c, field, dst, elems, stream);
    if (st) b->err = c->err;
    return st;
}

snowlb_status snowlb_batch_diag(snowlb_batch* b, int32_t i, double* out, void* stream) {
    if (!b || i < 0 || i >= (int32_t)b->doms.size()) return SNOWLB_EINVAL;
    snowlb_ctx* c = b->doms[i];
    c->drv.par = b->drv.par;
    c->drv.step = b->drv.step;
    snowlb_status st = snowlb_diag(c, out, stream);
    if (st) b->err = c->err;
    return st;
}

snowlb_status snowlb_batch_set_tile(snowlb_batch* b, int32_t tile, int32_t mode) {
    if (!b) return SNOWLB_EINVAL;
    if (tile < 0 || tile >= tile_config_count() || mode < 0 || mode >= kLaunchModes) {
        b->err = "unknown tile configuration or grid mode";
        return SNOWLB_EINVAL;
    }
    b->drv.tile = tile;
    b->drv.grid_mode = mode;
    b->tuned = true;
    b->drv.drop_graph();
    return SNOWLB_OK;
}

int32_t snowlb_batch_get_tile(const snowlb_batch* b) { return b ? b->drv.tile : -1; }

snowlb_status snowlb_bw_probe(void* dst, const void* src, int64_t bytes, void* stream) {
    if (!dst || !src || bytes < 0 || bytes % 16) return fail(nullptr, SNOWLB_EINVAL, "bw_probe: bad arguments");
    hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "copy kernel");
    return SNOWLB_OK;
}

}  // extern "C"
