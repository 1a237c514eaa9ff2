// Host runtime behind include/ppo.h: argument validation (always before any
// enqueue), the flat parameter layout, workspace planning, the launch
// sequence of each entry point, and the cache of captured HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ppo.h"
#include "common.hpp"

using namespace ppo;

namespace {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(PPO_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define PPO_HIP(expr, what)                          \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_ptr(const void *p, const char *name, bool nullable = false) {
    if (!p) return nullable ? PPO_OK : fail(PPO_E_INVAL, "%s is NULL", name);
    if (!aligned16(p)) return fail(PPO_E_INVAL, "%s is not 16-byte aligned", name);
    return PPO_OK;
}

#define PPO_CHECK(expr)              \
    do {                             \
        int _rc = (expr);            \
        if (_rc != PPO_OK) return _rc; \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int cdiv(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }

// ------------------------------------------------------------- net layout
struct NetLayout {
    int L = 0;          // hidden layers
    int D = 0, A = 0;
    int H[kMaxHidden] = {0};
    int dims_a[kMaxLayers + 1] = {0};  // actor widths, input first
    int dims_c[kMaxLayers + 1] = {0};
    long long Wa[kMaxLayers] = {0}, ba[kMaxLayers] = {0};
    long long Wc[kMaxLayers] = {0}, bc[kMaxLayers] = {0};
    long long logstd = 0, P = 0;
};

int validate_net(const ppo_net_desc *net) {
    if (!net) return fail(PPO_E_INVAL, "net is NULL");
    if (net->obs_dim < 1 || net->obs_dim > PPO_MAX_OBS)
        return fail(PPO_E_SHAPE, "obs_dim %d outside 1..%d", net->obs_dim, PPO_MAX_OBS);
    if (net->act_dim < 1 || net->act_dim > PPO_MAX_ACT)
        return fail(PPO_E_SHAPE, "act_dim %d outside 1..%d", net->act_dim, PPO_MAX_ACT);
    if (net->n_hidden < 1 || net->n_hidden > PPO_MAX_HIDDEN)
        return fail(PPO_E_SHAPE, "n_hidden %d outside 1..%d", net->n_hidden, PPO_MAX_HIDDEN);
    for (int l = 0; l < net->n_hidden; ++l) {
        const int h = net->hidden[l];
        if (h < 16 || h > PPO_MAX_WIDTH || h % 16 != 0)
            return fail(PPO_E_SHAPE, "hidden[%d] = %d must be a multiple of 16 in 16..%d", l, h, PPO_MAX_WIDTH);
    }
    return PPO_OK;
}

NetLayout make_layout(const ppo_net_desc &net) {
    NetLayout g;
    g.L = net.n_hidden;
    g.D = net.obs_dim;
    g.A = net.act_dim;
    g.dims_a[0] = g.dims_c[0] = g.D;
    for (int l = 0; l < g.L; ++l) {
        g.H[l] = net.hidden[l];
        g.dims_a[l + 1] = g.dims_c[l + 1] = g.H[l];
    }
    g.dims_a[g.L + 1] = g.A;
    g.dims_c[g.L + 1] = 1;
    long long off = 0;
    for (int l = 0; l <= g.L; ++l) {
        g.Wa[l] = off;
        off += static_cast<long long>(g.dims_a[l + 1]) * g.dims_a[l];
        g.ba[l] = off;
        off += g.dims_a[l + 1];
    }
    g.logstd = off;
    off += g.A;
    for (int l = 0; l <= g.L; ++l) {
        g.Wc[l] = off;
        off += static_cast<long long>(g.dims_c[l + 1]) * g.dims_c[l];
        g.bc[l] = off;
        off += g.dims_c[l + 1];
    }
    g.P = off;
    return g;
}

// --------------------------------------------------------- workspace plan
struct Region {
    size_t off = 0, bytes = 0;
};

struct WsPlan {
    // rows of the GEMM chain
    int rows = 0;
    int kpad = 0;      // padded observation width of the gathered input
    size_t esz = 4;    // bytes per activation element
    Region xg;
    Region h_a[kMaxHidden], h_c[kMaxHidden];
    Region dz_a[kMaxHidden], dz_c[kMaxHidden];
    Region dzh_a, dzh_c;
    Region part, rowsum, loss_part, loss_sums, sumsq, gae_part;
    // staged weights (elements of the operand type): the first layer padded
    // to kpad columns when D is not a multiple of 8, and W_l^T for l >= 1
    Region wt;
    // bf16 weights of the fused pass in MFMA fragment order: W_l for every
    // hidden layer and W_l^T for l >= 1 (elements)
    Region frag;
    size_t frag_w[2][kMaxHidden] = {{0}}, frag_wt[2][kMaxHidden] = {{0}};
    bool pad_w0 = false;
    size_t wt_w0[2] = {0, 0};
    size_t wt_t[2][kMaxHidden] = {{0}};
    // bf16: the critic's hidden weights' residuals theta - bf16(theta), row-major
    // [H_l][K_l] (K_0 = kpad), the second B operand of its forward GEMMs
    size_t wt_lo[kMaxHidden] = {0};
    int max_splits = 1;
    size_t total = 0;
};

struct Alloc {
    size_t cur = 0;
    Region take(size_t bytes) {
        Region r;
        r.off = cur;
        r.bytes = bytes;
        cur = align_up(cur + bytes, 256);
        return r;
    }
};

int gemm_bk(Precision p) { return p == kBF16 ? GemmTile<uint16_t>::BK : GemmTile<float>::BK; }

// Output shape of the weight-gradient problem of layer l (0-based, l == L is
// the output layer) for one network.
void dw_shape(const NetLayout &g, bool actor, int l, int &rows, int &cols) {
    rows = actor ? g.dims_a[l + 1] : g.dims_c[l + 1];
    cols = l == 0 ? g.D : g.H[l - 1];
}

int dw_tiles(const NetLayout &g, int tile) {
    int tiles = 0;
    for (int net = 0; net < 2; ++net)
        for (int l = 0; l <= g.L; ++l) {
            int r, c;
            dw_shape(g, net == 0, l, r, c);
            tiles += cdiv(r, tile_rows(tile)) * cdiv(c, tile_cols(tile));
        }
    return tiles;
}

// Two workgroups are resident on each of 256 CUs.  A weight-gradient
// workgroup streams its k-range at a roughly fixed time per k-slab, so a
// launch takes (rounds of resident workgroups) x (slabs per workgroup):
// split into `rounds` half rounds (1: one workgroup per CU, 2: one full
// round, 4: two), never a partial extra one.  Fewer splits write fewer
// partials for the reduction to read.
constexpr int kResidentSlots = 512;

void dw_splits(const NetLayout &g, Precision prec, int M, int tile, int rounds, int &splits, int &kps) {
    const int bk = gemm_bk(prec);
    int s = std::max(1, rounds * (kResidentSlots / 2) / dw_tiles(g, tile));
    s = std::min(s, std::max(1, M / (2 * bk)));
    kps = cdiv(cdiv(M, s), bk) * bk;
    splits = cdiv(M, kps);
}

// Largest split count any tuning candidate may use (sizes the partials).
int dw_max_splits(const NetLayout &g, Precision prec, int M) {
    int best = 1;
    for (int t = 0; t < kNumTileShapes; ++t)
        for (int rounds : {1, 2, 4}) {
            int sp, kps;
            dw_splits(g, prec, M, t, rounds, sp, kps);
            best = std::max(best, sp);
        }
    return best;
}

WsPlan plan_workspace(const NetLayout &g, Precision prec, int N, int T, int M) {
    WsPlan w;
    w.esz = prec == kBF16 ? 2 : 4;
    w.kpad = static_cast<int>(align_up(g.D, 8));
    const int rows = std::max(N, M);
    w.rows = rows;
    Alloc a;
    w.xg = a.take(static_cast<size_t>(rows) * w.kpad * w.esz);
    for (int l = 0; l < g.L; ++l) {
        w.h_a[l] = a.take(static_cast<size_t>(rows) * g.H[l] * w.esz);
        w.h_c[l] = a.take(static_cast<size_t>(rows) * g.H[l] * w.esz);
    }
    const int mm = std::max(M, 1);
    for (int l = 0; l < g.L; ++l) {
        w.dz_a[l] = a.take(static_cast<size_t>(mm) * g.H[l] * w.esz);
        w.dz_c[l] = a.take(static_cast<size_t>(mm) * g.H[l] * w.esz);
    }
    w.dzh_a = a.take(static_cast<size_t>(mm) * kHeadPad * w.esz);
    w.dzh_c = a.take(static_cast<size_t>(mm) * kHeadPad * w.esz);
    w.max_splits = dw_max_splits(g, prec, mm);
    size_t part_floats = 0, rowsum_floats = 0;
    for (int net = 0; net < 2; ++net)
        for (int l = 0; l <= g.L; ++l) {
            int r, c;
            dw_shape(g, net == 0, l, r, c);
            part_floats += align_up(static_cast<size_t>(w.max_splits) * r * c, 64);
            rowsum_floats += align_up(static_cast<size_t>(w.max_splits) * r, 64);
        }
    w.part = a.take(part_floats * 4);
    w.rowsum = a.take(rowsum_floats * 4);
    w.loss_part = a.take(static_cast<size_t>(head_loss_blocks(mm)) * head_loss_partial_width(g.A) * 4);
    w.loss_sums = a.take(8 * 4);
    w.sumsq = a.take(static_cast<size_t>(1024) * 8);
    w.gae_part = a.take(static_cast<size_t>(gae_blocks(std::max(N, 1))) * 3 * 8);
    w.pad_w0 = g.D != w.kpad;
    size_t wt_elems = 0;
    for (int net = 0; net < 2; ++net) {
        if (w.pad_w0) {
            w.wt_w0[net] = wt_elems;
            wt_elems += align_up(static_cast<size_t>(g.H[0]) * w.kpad, 64);
        }
        for (int l = 1; l < g.L; ++l) {
            w.wt_t[net][l] = wt_elems;
            wt_elems += align_up(static_cast<size_t>(g.H[l - 1]) * g.H[l], 64);
        }
    }
    if (prec == kBF16)
        for (int l = 0; l < g.L; ++l) {
            w.wt_lo[l] = wt_elems;
            wt_elems += align_up(static_cast<size_t>(g.H[l]) * (l == 0 ? w.kpad : g.H[l - 1]), 64);
        }
    w.wt = a.take(std::max<size_t>(wt_elems, 1) * w.esz);
    size_t frag_elems = 0;
    if (prec == kBF16 && w.kpad % 16 == 0) {
        for (int net = 0; net < 2; ++net)
            for (int l = 0; l < g.L; ++l) {
                w.frag_w[net][l] = frag_elems;
                // the critic's forward fragments in the split layout (twice the size)
                frag_elems += static_cast<size_t>(g.H[l]) * (l == 0 ? w.kpad : g.H[l - 1]) * (net == 1 ? 2 : 1);
                if (l >= 1) {
                    w.frag_wt[net][l] = frag_elems;
                    frag_elems += static_cast<size_t>(g.H[l - 1]) * g.H[l];
                }
            }
    }
    w.frag = a.take(std::max<size_t>(frag_elems, 1) * 2);
    (void)T;
    w.total = a.cur;
    return w;
}

// -------------------------------------------------- packed-weight cache
// Inference reads the forward weights of a bf16 network in fragment order,
// packed from the shadow into the workspace.  Over a rollout the shadow does
// not change, so with PPO_OPT_KEEP_PACKED set on the context the pack is
// skipped when the workspace still holds the fragments of the same shadow at
// the same generation (the caller keeps its workspaces alive and writes them
// only through this library).  Host-side records, process-wide:
//   g_shadow_gen  per shadow, bumped by every write to it that this library
//                 enqueues; -1 (never trusted again) once such a write was
//                 enqueued under stream capture, since each replay of the
//                 captured work writes it again without passing through here;
//   g_frag_cache  which workspace ranges hold which (context, shadow,
//                 generation, offset) forward fragments; dropped by every
//                 other call whose workspace range overlaps.
// Packing under stream capture always packs and records nothing.
struct FragRecord {
    uintptr_t lo, hi;
    const ppo_ctx *ctx;
    const uint16_t *shadow;
    long long gen;
    size_t off;
};
std::mutex g_cache_mu;
std::map<const uint16_t *, long long> g_shadow_gen;
std::vector<FragRecord> g_frag_cache;

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    // an error counts as capturing: nothing is cached then
    return hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone;
}

void drop_overlapping(const void *ws, size_t bytes) {
    const uintptr_t lo = reinterpret_cast<uintptr_t>(ws), hi = lo + bytes;
    for (size_t i = 0; i < g_frag_cache.size();) {
        if (g_frag_cache[i].lo < hi && lo < g_frag_cache[i].hi)
            g_frag_cache.erase(g_frag_cache.begin() + static_cast<long>(i));
        else
            ++i;
    }
}

void note_ws_used(const void *ws, size_t bytes) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    drop_overlapping(ws, bytes);
}

void note_shadow_written(const uint16_t *shadow, hipStream_t s) {
    if (!shadow) return;
    const bool cap = stream_capturing(s);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    long long &g = g_shadow_gen[shadow];
    if (cap)
        g = -1;
    else if (g >= 0)
        ++g;
}

bool frags_current(const ppo_ctx *c, const uint16_t *shadow, const void *ws, size_t off) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_shadow_gen.find(shadow);
    const long long gen = it == g_shadow_gen.end() ? 0 : it->second;
    if (gen < 0) return false;
    const uintptr_t lo = reinterpret_cast<uintptr_t>(ws);
    for (const FragRecord &r : g_frag_cache)
        if (r.lo == lo && r.ctx == c && r.shadow == shadow && r.gen == gen && r.off == off) return true;
    return false;
}

void note_frags_packed(const ppo_ctx *c, const uint16_t *shadow, const void *ws, size_t bytes, size_t off,
                       hipStream_t s) {
    const bool cap = stream_capturing(s);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    drop_overlapping(ws, bytes);
    if (cap) return;
    const long long gen = g_shadow_gen[shadow];
    if (gen < 0) return;
    const uintptr_t lo = reinterpret_cast<uintptr_t>(ws);
    g_frag_cache.push_back(FragRecord{lo, lo + bytes, c, shadow, gen, off});
}

// --------------------------------------------------------------- device
std::mutex g_dev_mu;
std::map<int, int> g_dev_ok;  // device -> PPO_OK or error code

int check_device() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev_ok.find(dev);
    if (it != g_dev_ok.end()) {
        if (it->second != PPO_OK) return fail(it->second, "device %d is not gfx950", dev);
        return PPO_OK;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    g_dev_ok[dev] = ok ? PPO_OK : PPO_E_UNSUPPORTED;
    if (!ok) return fail(PPO_E_UNSUPPORTED, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    return PPO_OK;
}

// ----------------------------------------------------------- tile choices
// GEMM launch sites of one mini-batch step (or one rollout step).
enum Site { kSiteFwd = 0, kSiteDx = kMaxHidden, kSiteDw = 2 * kMaxHidden, kNumSites = 2 * kMaxHidden + 1 };

struct TileChoice {
    int tile = kTile128x128;
    int rounds = 2;  // weight-gradient splits: half rounds of resident workgroups (1, 2 or 4)
};

struct Tuning {
    TileChoice site[kNumSites];
};

}  // namespace

// ------------------------------------------------------------------ context
struct ppo_ctx {
    ppo_net_desc net{};
    NetLayout g;
    Precision prec = kFP32;
    std::mutex mu;
    hipStream_t capture = nullptr;
    int capture_dev = -1;
    std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
    std::vector<std::vector<uint64_t>> graph_order;  // insertion order for eviction
    std::map<int, Tuning> tuned;                      // GEMM rows -> measured tile choices
    bool keep_packed = false;                         // PPO_OPT_KEEP_PACKED
};

namespace {

constexpr size_t kMaxGraphs = 16;

struct Weights {
    const void *W[2][kMaxLayers];  // [net][layer] GEMM operand pointers (T)
};

Weights gemm_weights(const ppo_ctx *c, const ppo_params *p) {
    Weights w{};
    const NetLayout &g = c->g;
    for (int l = 0; l <= g.L; ++l) {
        if (c->prec == kBF16) {
            w.W[0][l] = p->shadow + g.Wa[l];
            w.W[1][l] = p->shadow + g.Wc[l];
        } else {
            w.W[0][l] = p->theta + g.Wa[l];
            w.W[1][l] = p->theta + g.Wc[l];
        }
    }
    return w;
}

char *wsp(void *ws, const Region &r) { return static_cast<char *>(ws) + r.off; }

// Event pairs recorded on the launch stream around each kernel of a step.
struct Profiler {
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> ev;
    std::vector<int> phase;
    size_t used = 0;
    int reps = 1;               // back-to-back repetitions of each repeatable launch
    bool reduce_repeatable = true;
    // Launches that only read what earlier launches wrote give the same
    // result when repeated; Adam (and the reduction when it adapts the rate)
    // change state and run once.
    int reps_for(int ph) const {
        if (ph == PPO_PHASE_ADAM || (ph == PPO_PHASE_GRAD_REDUCE && !reduce_repeatable)) return 1;
        return reps;
    }
    hipError_t begin(int ph) {
        while (ev.size() < used + 2) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev.push_back(e);
        }
        phase.push_back(ph);
        return hipEventRecord(ev[used], s);
    }
    hipError_t end() {
        hipError_t r = hipEventRecord(ev[used + 1], s);
        used += 2;
        return r;
    }
    ~Profiler() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

// Wraps one launch expression with profiling events when a profiler is set.
#define PROFILED(prof, ph, expr)                                  \
    do {                                                          \
        const int _reps = (prof) ? (prof)->reps_for(ph) : 1;      \
        if (prof) {                                               \
            hipError_t _pe = (prof)->begin(ph);                   \
            if (_pe != hipSuccess) return _pe;                    \
        }                                                         \
        for (int _r = 0; _r < _reps; ++_r) {                      \
            hipError_t _le = (expr);                              \
            if (_le != hipSuccess) return _le;                    \
        }                                                         \
        if (prof) {                                               \
            hipError_t _pe = (prof)->end();                       \
            if (_pe != hipSuccess) return _pe;                    \
        }                                                         \
    } while (0)

void add_problem(GemmArgs &args, const GemmProblem &proto, int bk) {
    GemmProblem p = proto;
    p.tiles_m = cdiv(p.M, tile_rows(args.tile));
    p.tiles_n = cdiv(p.N, tile_cols(args.tile));
    if (p.splits <= 0) {
        p.splits = 1;
        p.kps = cdiv(p.K, bk) * bk;
    }
    p.tile_begin = args.total_tiles;
    args.p[args.count++] = p;
    args.total_tiles += p.tiles_m * p.tiles_n * p.splits;
}

// Staged copies of the weights: the padded first layer (rollout and update)
// and, for the update, the transposed hidden layers W_1 .. W_{L-1}.
StageArgs build_stage(const ppo_ctx *c, const ppo_params *p, const WsPlan &w, void *ws, bool transposes) {
    const NetLayout &g = c->g;
    const Weights W = gemm_weights(c, p);
    StageArgs a{};
    char *base = static_cast<char *>(wsp(ws, w.wt));
    for (int net = 0; net < 2; ++net) {
        if (w.pad_w0) {
            StageJob j{};
            j.src = W.W[net][0];
            j.dst = base + w.wt_w0[net] * w.esz;
            j.rows = g.H[0];
            j.cols = g.D;
            j.src_ld = g.D;
            j.dst_ld = w.kpad;
            j.transpose = 0;
            add_stage_job(a, j);
        }
        if (net == 1 && c->prec == kBF16)
            for (int l = 0; l < g.L; ++l) {
                // the critic's weight residuals for the second pass of its forward GEMMs
                StageJob j{};
                j.lo_src = p->theta + g.Wc[l];
                j.dst = base + w.wt_lo[l] * w.esz;
                j.rows = g.H[l];
                j.cols = l == 0 ? g.D : g.H[l - 1];
                j.src_ld = j.cols;
                j.dst_ld = l == 0 ? w.kpad : j.cols;
                j.transpose = 0;
                add_stage_job(a, j);
            }
        if (!transposes) continue;
        for (int l = 1; l < g.L; ++l) {
            StageJob j{};
            j.src = W.W[net][l];
            j.dst = base + w.wt_t[net][l] * w.esz;
            j.rows = g.H[l];        // W_l is [H_l, H_{l-1}]
            j.cols = g.H[l - 1];
            j.src_ld = g.H[l - 1];
            j.dst_ld = g.H[l];      // W_l^T is [H_{l-1}, H_l]
            j.transpose = 1;
            add_stage_job(a, j);
        }
    }
    return a;
}

// Forward GEMM of hidden layer l for `rows` rows (input gathered in xg).
GemmArgs build_fwd(const ppo_ctx *c, const ppo_params *p, const WsPlan &w, void *ws, int rows, int l, bool actor,
                   bool critic, int tile) {
    const NetLayout &g = c->g;
    const Weights W = gemm_weights(c, p);
    GemmArgs args{};
    args.tile = tile;
    for (int net = 0; net < 2; ++net) {
        if ((net == 0 && !actor) || (net == 1 && !critic)) continue;
        GemmProblem q{};
        q.A = l == 0 ? static_cast<const void *>(wsp(ws, w.xg))
                     : static_cast<const void *>(wsp(ws, net == 0 ? w.h_a[l - 1] : w.h_c[l - 1]));
        q.lda = l == 0 ? w.kpad : g.H[l - 1];
        q.K = l == 0 ? g.D : g.H[l - 1];
        q.B = W.W[net][l];
        q.ldb = q.K;
        if (l == 0 && w.pad_w0) {
            // zero-padded copy: K runs over the padded width (zeros on both sides)
            q.B = static_cast<char *>(wsp(ws, w.wt)) + w.wt_w0[net] * w.esz;
            q.K = w.kpad;
            q.ldb = w.kpad;
        }
        if (net == 1 && c->prec == kBF16)
            q.B2 = static_cast<char *>(wsp(ws, w.wt)) + w.wt_lo[l] * w.esz;   // same layout and ld as B
        q.C = wsp(ws, net == 0 ? w.h_a[l] : w.h_c[l]);
        q.ldc = g.H[l];
        q.bias = p->theta + (net == 0 ? g.ba[l] : g.bc[l]);
        q.M = rows;
        q.N = g.H[l];
        add_problem(args, q, gemm_bk(c->prec));
    }
    return args;
}

// Input-gradient GEMM: dz_{l-1} = (dz_l W_l) * ELU'(z_{l-1}) for both
// networks, with W_l^T staged row-major (both operands k-contiguous).
GemmArgs build_dx(const ppo_ctx *c, const ppo_params *p, const WsPlan &w, void *ws, int M, int l, int tile) {
    const NetLayout &g = c->g;
    (void)p;
    GemmArgs args{};
    args.tile = tile;
    for (int net = 0; net < 2; ++net) {
        GemmProblem q{};
        q.A = wsp(ws, net == 0 ? w.dz_a[l] : w.dz_c[l]);
        q.lda = g.H[l];
        q.K = g.H[l];
        q.B = static_cast<char *>(wsp(ws, w.wt)) + w.wt_t[net][l] * w.esz;
        q.ldb = g.H[l];
        q.C = wsp(ws, net == 0 ? w.dz_a[l - 1] : w.dz_c[l - 1]);
        q.ldc = g.H[l - 1];
        q.H = wsp(ws, net == 0 ? w.h_a[l - 1] : w.h_c[l - 1]);
        q.ldh = g.H[l - 1];
        q.M = M;
        q.N = g.H[l - 1];
        add_problem(args, q, gemm_bk(c->prec));
    }
    return args;
}

// Weight-gradient GEMMs of every layer of both networks (split over the
// samples) and the gradient segments that sum their partials.
struct DwPlan {
    GemmArgs launch[2];
    int n_launch = 0;
    ReduceArgs red{};
};

// kps_layer (optional, per layer 0..L, both networks): samples per split in
// place of the run's own choice where positive.  Problems are added network
// by network, layer by layer: problem net * (L + 1) + l.
DwPlan build_dw(const ppo_ctx *c, const WsPlan &w, void *ws, int M, const TileChoice &tc,
                const int *kps_layer = nullptr) {
    const NetLayout &g = c->g;
    const int L = g.L;
    DwPlan d;
    int splits0, kps0;
    dw_splits(g, c->prec, M, tc.tile, tc.rounds, splits0, kps0);
    long long pos = 0;
    float *part = reinterpret_cast<float *>(wsp(ws, w.part));
    float *rows_part = reinterpret_cast<float *>(wsp(ws, w.rowsum));
    size_t part_off = 0, row_off = 0;
    d.launch[0] = GemmArgs{};
    d.launch[0].tile = tc.tile;
    for (int net = 0; net < 2; ++net) {
        for (int l = 0; l <= L; ++l) {
            int r, cc;
            dw_shape(g, net == 0, l, r, cc);
            int kps = kps0, splits = splits0;
            if (kps_layer && kps_layer[l] > 0) {
                kps = kps_layer[l];
                splits = cdiv(M, kps);
            }
            GemmProblem q{};
            if (l == L) {
                q.A = wsp(ws, net == 0 ? w.dzh_a : w.dzh_c);
                q.lda = kHeadPad;
            } else {
                q.A = wsp(ws, net == 0 ? w.dz_a[l] : w.dz_c[l]);
                q.lda = g.H[l];
            }
            if (l == 0) {
                q.B = wsp(ws, w.xg);
                q.ldb = w.kpad;
            } else {
                q.B = wsp(ws, net == 0 ? w.h_a[l - 1] : w.h_c[l - 1]);
                q.ldb = g.H[l - 1];
            }
            q.M = r;
            q.N = cc;
            q.K = M;
            q.C = part + part_off;
            q.ldc = cc;
            q.c_split_stride = static_cast<long long>(r) * cc;
            q.rowsum = rows_part + row_off;
            q.splits = splits;
            q.kps = kps;
            GemmArgs &cur = d.launch[d.n_launch];
            add_problem(cur, q, gemm_bk(c->prec));
            if (cur.count == kGemmMaxProblems && !(net == 1 && l == L)) {
                ++d.n_launch;
                d.launch[d.n_launch] = GemmArgs{};
                d.launch[d.n_launch].tile = tc.tile;
            }

            const long long woff = net == 0 ? g.Wa[l] : g.Wc[l];
            const long long boff = net == 0 ? g.ba[l] : g.bc[l];
            d.red.seg[d.red.count++] = ReduceSegment{part + part_off, static_cast<long long>(r) * cc, splits, r, cc,
                                                     cc, woff, pos, 0.0f};
            pos += static_cast<long long>(r) * cc;
            d.red.seg[d.red.count++] = ReduceSegment{rows_part + row_off, r, splits, 1, r, 0, boff, pos, 0.0f};
            pos += r;
            part_off += align_up(static_cast<size_t>(splits) * r * cc, 64);
            row_off += align_up(static_cast<size_t>(splits) * r, 64);
        }
    }
    ++d.n_launch;
    d.red.total = pos;
    return d;
}

// ------------------------------------------------------------- autotuner
// Each GEMM launch site picks its tile shape (and, for the weight
// gradients, its split rounds) by timing every candidate with HIP events on
// the caller's stream the first time a row count is seen.  Candidates touch
// only the workspace regions they would write anyway, so the timing launches
// leave no trace.  Results are kept per context and row count, and in the
// file named by PPO_TUNE_CACHE if set; PPO_AUTOTUNE=0 keeps the defaults.
std::mutex g_tune_file_mu;

std::string tune_key(const ppo_ctx *c, int rows, bool update) {
    std::string k = std::string(c->prec == kBF16 ? "bf16" : "fp32") + "|" + std::to_string(c->g.D) + "|" +
                    std::to_string(c->g.A) + "|";
    for (int l = 0; l < c->g.L; ++l) k += std::to_string(c->g.H[l]) + ",";
    k += "|" + std::to_string(rows) + (update ? "|u" : "|r") + "|2";
    return k;
}

bool tune_file_lookup(const std::string &key, Tuning &t) {
    const char *path = std::getenv("PPO_TUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_tune_file_mu);
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[512];
        int n = 0;
        if (std::sscanf(line, "%511s%n", k, &n) != 1 || key != k) continue;
        const char *q = line + n;
        Tuning tmp;
        bool ok = true;
        for (int i = 0; i < kNumSites && ok; ++i) {
            int used = 0;
            ok = std::sscanf(q, "%d %d%n", &tmp.site[i].tile, &tmp.site[i].rounds, &used) == 2 &&
                 tmp.site[i].tile >= 0 && tmp.site[i].tile < kNumTileShapes &&
                 (tmp.site[i].rounds == 1 || tmp.site[i].rounds == 2 || tmp.site[i].rounds == 4);
            q += used;
        }
        if (ok) {
            t = tmp;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_file_store(const std::string &key, const Tuning &t) {
    const char *path = std::getenv("PPO_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_tune_file_mu);
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s", key.c_str());
    for (int i = 0; i < kNumSites; ++i) std::fprintf(f, " %d %d", t.site[i].tile, t.site[i].rounds);
    std::fprintf(f, "\n");
    std::fclose(f);
}

// Median-free small timing: one warm-up launch, then `reps` launches between
// two events.
template <typename F>
hipError_t time_launch(hipStream_t s, F &&launch, int reps, float &ms) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

bool autotune_enabled() {
    const char *v = std::getenv("PPO_AUTOTUNE");
    return !(v && std::strcmp(v, "0") == 0);
}

// Tile choices for `rows` GEMM rows; `update` adds the input- and
// weight-gradient sites.  grad_scratch: a [P] float buffer the caller is
// about to overwrite (the step's gradient), into which the weight-gradient
// candidates are reduced while they are timed; null times the GEMMs alone.
// Must not be called while the stream is captured.
int ensure_tuned(const ppo_ctx *cc, const ppo_params *p, const WsPlan &w, void *ws, int rows, bool update,
                 hipStream_t s, Tuning &out, float *grad_scratch = nullptr) {
    ppo_ctx *c = const_cast<ppo_ctx *>(cc);
    const int key_rows = update ? -rows : rows;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->tuned.find(key_rows);
        if (it != c->tuned.end()) {
            out = it->second;
            return PPO_OK;
        }
    }
    Tuning t;
    const std::string key = tune_key(c, rows, update);
    if (autotune_enabled() && !tune_file_lookup(key, t)) {
        const NetLayout &g = c->g;
        const Precision prec = c->prec;
        const int reps = 3;
        for (int l = 0; l < g.L; ++l) {
            float best = 1e30f;
            for (int tile = 0; tile < kNumTileShapes; ++tile) {
                GemmArgs a = build_fwd(c, p, w, ws, rows, l, true, true, tile);
                float ms = 0.0f;
                PPO_HIP(time_launch(s, [&] { return launch_gemm(prec, 0, 0, kEpiBiasElu, a, s); }, reps, ms),
                        "autotune forward");
                if (ms < best) {
                    best = ms;
                    t.site[kSiteFwd + l].tile = tile;
                }
            }
        }
        if (update) {
            for (int l = 1; l < g.L; ++l) {
                float best = 1e30f;
                for (int tile = 0; tile < kNumTileShapes; ++tile) {
                    GemmArgs a = build_dx(c, p, w, ws, rows, l, tile);
                    float ms = 0.0f;
                    PPO_HIP(time_launch(s, [&] { return launch_gemm(prec, 0, 0, kEpiDElu, a, s); }, reps, ms),
                            "autotune input gradient");
                    if (ms < best) {
                        best = ms;
                        t.site[kSiteDx + l].tile = tile;
                    }
                }
            }
            // each candidate is timed with the reduction of its partials (no
            // rate update), since fewer splits trade GEMM parallelism for
            // fewer partial bytes
            float best = 1e30f;
            for (int tile = 0; tile < kNumTileShapes; ++tile)
                for (int rounds : {1, 2, 4}) {
                    TileChoice tc;
                    tc.tile = tile;
                    tc.rounds = rounds;
                    DwPlan d = build_dw(c, w, ws, rows, tc);
                    ReduceArgs &red = d.red;
                    red.grad = grad_scratch;
                    red.sumsq_partials = reinterpret_cast<double *>(wsp(ws, w.sumsq));
                    red.loss_partials = reinterpret_cast<const float *>(wsp(ws, w.loss_part));
                    red.n_loss = head_loss_blocks(rows);
                    red.loss_width = head_loss_partial_width(g.A);
                    red.A = g.A;
                    red.logstd_offset = g.logstd;
                    red.loss_sums = reinterpret_cast<float *>(wsp(ws, w.loss_sums));
                    red.inv_m = 1.0f / static_cast<float>(rows);
                    red.lr = nullptr;
                    float ms = 0.0f;
                    PPO_HIP(time_launch(
                                s,
                                [&] {
                                    hipError_t r = hipSuccess;
                                    for (int i = 0; i < d.n_launch && r == hipSuccess; ++i)
                                        r = launch_gemm(prec, 1, 1, kEpiPartial, d.launch[i], s);
                                    if (r == hipSuccess && grad_scratch) r = launch_grad_reduce(red, s);
                                    return r;
                                },
                                reps, ms),
                            "autotune weight gradient");
                    if (ms < best) {
                        best = ms;
                        t.site[kSiteDw] = tc;
                    }
                }
        }
        tune_file_store(key, t);
    }
    std::lock_guard<std::mutex> lk(c->mu);
    c->tuned[key_rows] = t;
    out = t;
    return PPO_OK;
}

// Forward through the hidden layers of the selected networks for `rows`
// rows whose gathered input is already in the xg region.
hipError_t enqueue_forward(const ppo_ctx *c, const ppo_params *p, const WsPlan &w, void *ws, int rows,
                           bool actor, bool critic, const Tuning &t, hipStream_t s, Profiler *prof = nullptr) {
    for (int l = 0; l < c->g.L; ++l) {
        const GemmArgs args = build_fwd(c, p, w, ws, rows, l, actor, critic, t.site[kSiteFwd + l].tile);
        PROFILED(prof, PPO_PHASE_FORWARD, launch_gemm(c->prec, 0, 0, kEpiBiasElu, args, s));
    }
    return hipSuccess;
}

struct StepBuffers {
    const ppo_batch *b;
    const int32_t *idx;  // M rows of this step
    int M;
    float *grad;         // destination of the assembled gradient
    float *stats;        // [kStatsWidth]
    int apply;           // Adam step or statistics only
    int step_offset;
    bool frags_ready = false;   // the fused pass's fragments already hold the current shadow
    bool write_frags = false;   // Adam refreshes them for the next step
    uint8_t *active_out = nullptr;  // per-sample surrogate branch (ppo_loss_grad only)
    bool loss_only = false;         // ppo_loss_grad without a gradient output
    float *ratio_out = nullptr;     // per-sample probability ratio (ppo_loss_grad only)
};

// Head/loss arguments of one mini-batch step over the rows idx[0 .. M).
HeadLossArgs head_loss_args(const ppo_ctx *c, const ppo_params *p, const ppo_hparams *hp, const WsPlan &w,
                            void *ws, const ppo_batch *b, const int32_t *idx, int M) {
    const NetLayout &g = c->g;
    const int L = g.L;
    HeadLossArgs hl{};
    hl.ha = wsp(ws, w.h_a[L - 1]);
    hl.hc = wsp(ws, w.h_c[L - 1]);
    hl.Wa = p->theta + g.Wa[L];
    hl.ba = p->theta + g.ba[L];
    hl.logstd = p->theta + g.logstd;
    hl.Wc = p->theta + g.Wc[L];
    hl.bc = p->theta + g.bc[L];
    hl.actions = b->actions;
    hl.logp_old = b->logp;
    hl.adv = b->adv;
    hl.returns = b->returns;
    hl.values_old = b->values;
    hl.mu_old = b->mu_old;
    hl.logstd_old = b->mu_old ? b->logstd_old : nullptr;
    hl.idx = idx;
    hl.B = b->B;
    hl.dza = wsp(ws, w.dz_a[L - 1]);
    hl.dzc = wsp(ws, w.dz_c[L - 1]);
    hl.dz_head_a = wsp(ws, w.dzh_a);
    hl.dz_head_c = wsp(ws, w.dzh_c);
    hl.partials = reinterpret_cast<float *>(wsp(ws, w.loss_part));
    hl.M = M;
    hl.A = g.A;
    hl.Hl = g.H[L - 1];
    hl.clip = hp->clip;
    hl.value_coef = hp->value_coef;
    hl.inv_m = 1.0f / static_cast<float>(M);
    hl.clip_value = hp->clip_value;
    return hl;
}

// The loss-partial half of the gradient assembly (the segments come from
// build_dw).  The learning rate adapts only in an optimiser step.
void set_reduce_loss(ReduceArgs &red, const ppo_ctx *c, const ppo_params *p, const ppo_hparams *hp,
                     const WsPlan &w, void *ws, float *grad, int M, int apply, int fused_r = 0) {
    const NetLayout &g = c->g;
    red.grad = grad;
    red.sumsq_partials = reinterpret_cast<double *>(wsp(ws, w.sumsq));
    red.loss_partials = reinterpret_cast<const float *>(wsp(ws, w.loss_part));
    red.n_loss = fused_r > 0 ? fused_blocks(M, fused_r) : head_loss_blocks(M);
    red.loss_width = head_loss_partial_width(g.A);
    red.A = g.A;
    red.logstd_offset = g.logstd;
    red.entropy_coef = hp->entropy_coef;
    red.loss_sums = reinterpret_cast<float *>(wsp(ws, w.loss_sums));
    red.inv_m = 1.0f / static_cast<float>(M);
    red.lr = apply && hp->desired_kl > 0.0f ? p->lr : nullptr;
    red.desired_kl = hp->desired_kl;
    red.lr_factor = hp->lr_factor;
    red.lr_min = hp->lr_min;
    red.lr_max = hp->lr_max;
}

AdamArgs adam_args(const ppo_ctx *c, const ppo_params *p, const ppo_hparams *hp, const ReduceArgs &red,
                   float *grad, float *stats, int M, int step_offset, int apply) {
    AdamArgs ad{};
    ad.theta = p->theta;
    ad.grad = grad;
    ad.m = p->adam_m;
    ad.v = p->adam_v;
    ad.shadow = c->prec == kBF16 ? p->shadow : nullptr;
    ad.step = p->step;
    ad.step_offset = step_offset;
    ad.lr = p->lr;
    ad.sumsq_partials = red.sumsq_partials;
    ad.n_sumsq = reduce_blocks(red.total);
    ad.loss_sums = red.loss_sums;
    ad.max_grad_norm = hp->max_grad_norm;
    ad.beta1 = hp->beta1;
    ad.beta2 = hp->beta2;
    ad.eps = hp->adam_eps;
    ad.inv_m = 1.0f / static_cast<float>(M);
    ad.value_coef = hp->value_coef;
    ad.entropy_coef = hp->entropy_coef;
    ad.stats = stats;
    ad.P = c->g.P;
    ad.apply = apply;
    return ad;
}

bool fused_env_enabled() {
    const char *v = std::getenv("PPO_FUSED");
    return !(v && std::strcmp(v, "0") == 0);
}


// Shape of the fused per-sample pass for this step, or rows = 0 for the
// layer-by-layer kernels: bf16 only, a network shape the fused kernel
// covers, 16-byte aligned biases, and observation offsets that fit its
// 32-bit buffer addressing.  PPO_FUSED=0 forces the layer-by-layer path;
// PPO_FUSED_ROWS and PPO_FUSED_THREADS restrict the block shape.
FusedShape fused_shape_for(const ppo_ctx *c, const ppo_params *p, const WsPlan &w, int obs_rows,
                           bool inference = false) {
    const FusedShape none{0, 0, 0};
    if (c->prec != kBF16 || !fused_env_enabled()) return none;
    const NetLayout &g = c->g;
    const char *rows = std::getenv("PPO_FUSED_ROWS");
    const char *threads = std::getenv("PPO_FUSED_THREADS");
    const char *per_cu = inference ? nullptr : std::getenv("PPO_FUSED_PER_CU");
    FusedShape sh = fused_shape(g.L, g.H, w.kpad, g.A, rows ? std::atoi(rows) : 0, threads ? std::atoi(threads) : 0,
                                !inference, per_cu ? std::atoi(per_cu) : 0);
    if (sh.rows == 0) return none;
    if (static_cast<long long>(obs_rows) * g.D * 4 > 0x7FFFFFF0LL - 0x100000LL) return none;
    for (int net = 0; net < 2; ++net)
        for (int l = 0; l < g.L; ++l)
            if (!aligned16(p->theta + (net == 0 ? g.ba[l] : g.bc[l]))) return none;
    return sh;
}

// Packing of the bf16 shadow weights into fragment order for the fused pass.
FragArgs build_frags(const ppo_ctx *c, const ppo_params *p, const WsPlan &w, void *ws, bool transposes = true) {
    const NetLayout &g = c->g;
    const Weights W = gemm_weights(c, p);
    uint16_t *base = reinterpret_cast<uint16_t *>(wsp(ws, w.frag));
    FragArgs a{};
    for (int net = 0; net < 2; ++net)
        for (int l = 0; l < g.L; ++l) {
            const int K = l == 0 ? g.D : g.H[l - 1];
            FragJob j{};
            j.src = static_cast<const uint16_t *>(W.W[net][l]);
            j.dst = base + w.frag_w[net][l];
            j.rows = g.H[l];
            j.K = K;
            j.S = (l == 0 ? w.kpad : K) / 16;
            j.ld = K;
            j.transpose = 0;
            if (net == 1) {
                // the critic's forward weights: bf16 value and residual from theta
                j.split = 1;
                j.src32 = p->theta + g.Wc[l];
            }
            add_frag_job(a, j);
            if (l >= 1 && transposes) {
                FragJob t{};
                t.src = static_cast<const uint16_t *>(W.W[net][l]);
                t.dst = base + w.frag_wt[net][l];
                t.rows = g.H[l - 1];
                t.K = g.H[l];
                t.S = g.H[l] / 16;
                t.ld = g.H[l - 1];
                t.transpose = 1;
                add_frag_job(a, t);
            }
        }
    return a;
}

// The fragment copies of every hidden-layer weight of both networks (the
// same layouts and places as build_frags), for Adam to refresh.
void add_adam_frags(AdamArgs &ad, const ppo_ctx *c, const WsPlan &w, void *ws) {
    const NetLayout &g = c->g;
    uint16_t *base = reinterpret_cast<uint16_t *>(wsp(ws, w.frag));
    ad.n_frag = 0;
    for (int net = 0; net < 2; ++net)
        for (int l = 0; l < g.L; ++l) {
            AdamFrag &F = ad.frag[ad.n_frag++];
            F.begin = net == 0 ? g.Wa[l] : g.Wc[l];
            F.rows = g.H[l];
            F.cols = l == 0 ? g.D : g.H[l - 1];
            F.S = (l == 0 ? w.kpad : F.cols) / 16;
            F.S_t = g.H[l] / 16;
            F.split = net == 1 ? 1 : 0;
            F.dst = base + w.frag_w[net][l];
            F.dst_t = l >= 1 ? base + w.frag_wt[net][l] : nullptr;
        }
}

FusedArgs fused_args(const ppo_ctx *c, const ppo_params *p, const ppo_hparams *hp, const WsPlan &w, void *ws,
                     const ppo_batch *b, const int32_t *idx, int M) {
    const NetLayout &g = c->g;
    const uint16_t *frag = reinterpret_cast<const uint16_t *>(wsp(ws, w.frag));
    FusedArgs a{};
    for (int net = 0; net < 2; ++net) {
        FusedNet &n = a.net[net];
        for (int l = 0; l < g.L; ++l) {
            n.W[l] = frag + w.frag_w[net][l];
            n.WT[l] = l >= 1 ? frag + w.frag_wt[net][l] : nullptr;
            n.bias[l] = p->theta + (net == 0 ? g.ba[l] : g.bc[l]);
            n.h[l] = reinterpret_cast<uint16_t *>(wsp(ws, net == 0 ? w.h_a[l] : w.h_c[l]));
            n.dz[l] = reinterpret_cast<uint16_t *>(wsp(ws, net == 0 ? w.dz_a[l] : w.dz_c[l]));
        }
        n.dzh = reinterpret_cast<uint16_t *>(wsp(ws, net == 0 ? w.dzh_a : w.dzh_c));
        n.Wout = p->theta + (net == 0 ? g.Wa[g.L] : g.Wc[g.L]);
        n.bout = p->theta + (net == 0 ? g.ba[g.L] : g.bc[g.L]);
    }
    a.L = g.L;
    a.D = g.D;
    a.kpad = w.kpad;
    a.A = g.A;
    for (int l = 0; l < g.L; ++l) a.H[l] = g.H[l];
    a.obs = b->obs;
    a.idx = idx;
    a.B = b->B;
    a.M = M;
    a.actions = b->actions;
    a.logp_old = b->logp;
    a.adv = b->adv;
    a.returns = b->returns;
    a.values_old = b->values;
    a.mu_old = b->mu_old;
    a.logstd_old = b->mu_old ? b->logstd_old : nullptr;
    a.logstd = p->theta + g.logstd;
    a.xg = reinterpret_cast<uint16_t *>(wsp(ws, w.xg));
    a.partials = reinterpret_cast<float *>(wsp(ws, w.loss_part));
    a.clip = hp->clip;
    a.value_coef = hp->value_coef;
    a.inv_m = 1.0f / static_cast<float>(M);
    a.clip_value = hp->clip_value;
    return a;
}

// One mini-batch step: gather, forward, head+loss, input-gradient chain,
// weight gradients, gradient assembly with the float64 norm, Adam.
hipError_t enqueue_step(const ppo_ctx *c, const ppo_params *p, const ppo_hparams *hp, const WsPlan &w, void *ws,
                        const StepBuffers &sb, const Tuning &t, hipStream_t s, Profiler *prof = nullptr) {
    const NetLayout &g = c->g;
    const Precision prec = c->prec;
    const int M = sb.M;
    const int L = g.L;
    hipError_t e;

    const FusedShape fsh = fused_shape_for(c, p, w, sb.b->B);
    const int fused_r = fsh.rows;
    if (fused_r > 0) {
        // weights into fragment order, then gather, forward, loss and input
        // gradients of both networks in one launch
        if (!sb.frags_ready) PROFILED(prof, PPO_PHASE_GATHER, launch_pack_frags(build_frags(c, p, w, ws), s));
        FusedArgs fa = fused_args(c, p, hp, w, ws, sb.b, sb.idx, M);
        fa.active_out = sb.active_out;
        fa.no_backward = sb.loss_only ? 1 : 0;
        fa.ratio_out = sb.ratio_out;
        fa.R = fsh.rows;
        fa.NT = fsh.threads;
        fa.per_cu = fsh.per_cu;
        PROFILED(prof, PPO_PHASE_FUSED, launch_fused_update(fa, s));
    } else {
        PROFILED(prof, PPO_PHASE_GATHER, launch_stage_weights(prec, build_stage(c, p, w, ws, true), s));
        PROFILED(prof, PPO_PHASE_GATHER, launch_gather_obs(prec, s, sb.b->obs, sb.idx, sb.b->B, M, g.D, w.kpad,
                                                           wsp(ws, w.xg)));
        e = enqueue_forward(c, p, w, ws, M, true, true, t, s, prof);
        if (e != hipSuccess) return e;

        HeadLossArgs hl = head_loss_args(c, p, hp, w, ws, sb.b, sb.idx, M);
        hl.active_out = sb.active_out;
        hl.ratio_out = sb.ratio_out;
        PROFILED(prof, PPO_PHASE_HEAD_LOSS, launch_head_loss(prec, hl, s));

        for (int l = L - 1; l >= 1 && !sb.loss_only; --l) {
            const GemmArgs args = build_dx(c, p, w, ws, M, l, t.site[kSiteDx + l].tile);
            PROFILED(prof, PPO_PHASE_INPUT_GRAD, launch_gemm(prec, 0, 0, kEpiDElu, args, s));
        }
    }

    DwPlan d{};
    if (!sb.loss_only) {
        d = build_dw(c, w, ws, M, t.site[kSiteDw]);
        for (int i = 0; i < d.n_launch; ++i)
            PROFILED(prof, PPO_PHASE_WEIGHT_GRAD, launch_gemm(prec, 1, 1, kEpiPartial, d.launch[i], s));
    }

    ReduceArgs &red = d.red;
    set_reduce_loss(red, c, p, hp, w, ws, sb.grad, M, sb.apply, fused_r);
    PROFILED(prof, PPO_PHASE_GRAD_REDUCE, launch_grad_reduce(red, s));

    AdamArgs ad = adam_args(c, p, hp, red, sb.grad, sb.stats, M, sb.step_offset, sb.apply);
    if (fused_r > 0 && sb.write_frags && sb.apply) add_adam_frags(ad, c, w, ws);
    PROFILED(prof, PPO_PHASE_ADAM, launch_adam(ad, s));
    return hipSuccess;
}

int validate_hparams(const ppo_hparams *hp) {
    if (!hp) return fail(PPO_E_INVAL, "hparams is NULL");
    if (!(hp->clip > 0.0f) || !(hp->value_coef >= 0.0f) || !(hp->entropy_coef >= 0.0f) ||
        !(hp->max_grad_norm > 0.0f) || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) ||
        !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) || !(hp->adam_eps > 0.0f))
        return fail(PPO_E_INVAL, "hyper-parameter out of range");
    if (hp->clip_value != 0 && hp->clip_value != 1) return fail(PPO_E_INVAL, "clip_value must be 0 or 1");
    if (hp->use_graph != 0 && hp->use_graph != 1) return fail(PPO_E_INVAL, "use_graph must be 0 or 1");
    if (!(hp->desired_kl >= 0.0f) || !std::isfinite(hp->desired_kl))
        return fail(PPO_E_INVAL, "desired_kl must be finite and >= 0");
    if (hp->desired_kl > 0.0f &&
        (!(hp->lr_factor >= 1.0f) || !std::isfinite(hp->lr_factor) || !(hp->lr_min > 0.0f) ||
         !(hp->lr_max >= hp->lr_min) || !std::isfinite(hp->lr_max)))
        return fail(PPO_E_INVAL, "adaptive rate needs lr_factor >= 1 and 0 < lr_min <= lr_max");
    return PPO_OK;
}

int validate_params(const ppo_ctx *c, const ppo_params *p, bool need_optimizer) {
    if (!p) return fail(PPO_E_INVAL, "params is NULL");
    PPO_CHECK(check_ptr(p->theta, "params.theta"));
    if (c->prec == kBF16) PPO_CHECK(check_ptr(p->shadow, "params.shadow"));
    if (need_optimizer) {
        PPO_CHECK(check_ptr(p->grad, "params.grad"));
        PPO_CHECK(check_ptr(p->adam_m, "params.adam_m"));
        PPO_CHECK(check_ptr(p->adam_v, "params.adam_v"));
        if (!p->step) return fail(PPO_E_INVAL, "params.step is NULL");
        if (!p->lr) return fail(PPO_E_INVAL, "params.lr is NULL");
    }
    return PPO_OK;
}

int validate_batch(const ppo_ctx *c, const ppo_batch *b, const ppo_hparams *hp) {
    if (!b) return fail(PPO_E_INVAL, "batch is NULL");
    if (b->B < 1) return fail(PPO_E_SHAPE, "batch.B = %d must be positive", b->B);
    PPO_CHECK(check_ptr(b->obs, "batch.obs"));
    PPO_CHECK(check_ptr(b->actions, "batch.actions"));
    PPO_CHECK(check_ptr(b->logp, "batch.logp"));
    PPO_CHECK(check_ptr(b->adv, "batch.adv"));
    PPO_CHECK(check_ptr(b->returns, "batch.returns"));
    if (hp->clip_value) PPO_CHECK(check_ptr(b->values, "batch.values"));
    if (hp->desired_kl > 0.0f && !b->mu_old)
        return fail(PPO_E_INVAL, "desired_kl > 0 needs batch.mu_old and batch.logstd_old");
    if (b->mu_old) {
        PPO_CHECK(check_ptr(b->mu_old, "batch.mu_old"));
        if (!b->logstd_old) return fail(PPO_E_INVAL, "batch.logstd_old is NULL while batch.mu_old is set");
    }
    (void)c;
    return PPO_OK;
}

int validate_ws(const ppo_ctx *c, int N, int T, int M, const void *ws, size_t ws_bytes) {
    PPO_CHECK(check_ptr(ws, "ws"));
    const WsPlan w = plan_workspace(c->g, c->prec, N, T, M);
    if (ws_bytes < w.total)
        return fail(PPO_E_NOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, w.total);
    return PPO_OK;
}

int ensure_capture_stream(ppo_ctx *c) {
    int dev = 0;
    PPO_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (c->capture && c->capture_dev != dev) {
        // graphs and the capture stream belong to the previous device
        for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        c->graphs.clear();
        c->graph_order.clear();
        (void)hipStreamDestroy(c->capture);
        c->capture = nullptr;
    }
    if (!c->capture) {
        PPO_HIP(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking), "hipStreamCreate");
        c->capture_dev = dev;
    }
    return PPO_OK;
}

uint64_t u64(const void *p) { return static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p)); }
uint64_t fbits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

}  // namespace

// ================================================================ C ABI ====
extern "C" {

const char *ppo_last_error(void) { return g_error.c_str(); }

int ppo_param_count(const ppo_net_desc *net, int64_t *count) {
    PPO_CHECK(validate_net(net));
    if (!count) return fail(PPO_E_INVAL, "count is NULL");
    *count = make_layout(*net).P;
    return PPO_OK;
}

int ppo_param_offsets(const ppo_net_desc *net, int64_t *offsets, int32_t capacity) {
    PPO_CHECK(validate_net(net));
    if (!offsets) return fail(PPO_E_INVAL, "offsets is NULL");
    const NetLayout g = make_layout(*net);
    const int need = 4 * (g.L + 1) + 1;
    if (capacity < need) return fail(PPO_E_SHAPE, "offsets capacity %d < %d", capacity, need);
    int k = 0;
    for (int l = 0; l <= g.L; ++l) {
        offsets[k++] = g.Wa[l];
        offsets[k++] = g.ba[l];
    }
    offsets[k++] = g.logstd;
    for (int l = 0; l <= g.L; ++l) {
        offsets[k++] = g.Wc[l];
        offsets[k++] = g.bc[l];
    }
    return PPO_OK;
}

int ppo_ctx_create(const ppo_net_desc *net, int32_t precision, ppo_ctx **out) {
    PPO_CHECK(validate_net(net));
    if (!out) return fail(PPO_E_INVAL, "out is NULL");
    if (precision != PPO_FP32 && precision != PPO_BF16) return fail(PPO_E_INVAL, "precision %d", precision);
    ppo_ctx *c = new (std::nothrow) ppo_ctx();
    if (!c) return fail(PPO_E_INVAL, "out of host memory");
    c->net = *net;
    c->g = make_layout(*net);
    c->prec = precision == PPO_BF16 ? kBF16 : kFP32;
    *out = c;
    return PPO_OK;
}

int ppo_ctx_destroy(ppo_ctx *c) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (size_t i = 0; i < g_frag_cache.size();) {
            if (g_frag_cache[i].ctx == c)
                g_frag_cache.erase(g_frag_cache.begin() + static_cast<long>(i));
            else
                ++i;
        }
    }
    delete c;
    return PPO_OK;
}

int ppo_ctx_set_option(ppo_ctx *c, int32_t option, int32_t value) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    if (option != PPO_OPT_KEEP_PACKED) return fail(PPO_E_INVAL, "unknown option %d", option);
    if (value != 0 && value != 1) return fail(PPO_E_INVAL, "option value %d is not 0 or 1", value);
    c->keep_packed = value == 1;
    return PPO_OK;
}

int ppo_workspace_size(const ppo_ctx *c, int32_t N, int32_t T, int32_t M, size_t *bytes) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    if (!bytes) return fail(PPO_E_INVAL, "bytes is NULL");
    if (N < 0 || T < 0 || M < 0) return fail(PPO_E_SHAPE, "negative size");
    *bytes = plan_workspace(c->g, c->prec, N, T, M).total;
    return PPO_OK;
}

int ppo_pack_weights(const ppo_ctx *c, void *stream, const float *theta, uint16_t *shadow) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    PPO_CHECK(check_ptr(theta, "theta"));
    PPO_CHECK(check_ptr(shadow, "shadow"));
    PPO_CHECK(check_device());
    note_shadow_written(shadow, static_cast<hipStream_t>(stream));
    PPO_HIP(launch_pack_bf16(theta, shadow, c->g.P, static_cast<hipStream_t>(stream)), "pack_bf16");
    return PPO_OK;
}

int ppo_rollout_infer(const ppo_ctx *c, void *stream, const ppo_params *p, const float *obs, int32_t N, int32_t t,
                      uint64_t seed, uint32_t iteration, float *actions, float *logp, float *values, float *mu,
                      void *ws, size_t ws_bytes) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    if (N < 1) return fail(PPO_E_SHAPE, "N = %d must be positive", N);
    if (t < 0) return fail(PPO_E_SHAPE, "t = %d must be non-negative", t);
    PPO_CHECK(validate_params(c, p, false));
    PPO_CHECK(check_ptr(obs, "obs"));
    const bool value_only = actions == nullptr;
    PPO_CHECK(check_ptr(actions, "actions", true));
    PPO_CHECK(check_ptr(logp, "logp", true));
    PPO_CHECK(check_ptr(values, "values", !value_only));
    PPO_CHECK(check_ptr(mu, "mu", true));
    if (value_only && !values) return fail(PPO_E_INVAL, "value-only mode needs values");
    PPO_CHECK(validate_ws(c, N, 0, 0, ws, ws_bytes));
    PPO_CHECK(check_device());

    const hipStream_t s = static_cast<hipStream_t>(stream);
    const NetLayout &g = c->g;
    const WsPlan w = plan_workspace(g, c->prec, N, 0, 0);
    const FusedShape fsh = fused_shape_for(c, p, w, N, true);
    if (fsh.rows > 0) {
        // forward weights into fragment order, then one launch for the whole
        // forward pass and the sampling head
        // a captured call always packs: its replays may follow any shadow write
        if (!(c->keep_packed && !stream_capturing(s) && frags_current(c, p->shadow, ws, w.frag.off))) {
            PPO_HIP(launch_pack_frags(build_frags(c, p, w, ws, false), s), "pack_frags");
            note_frags_packed(c, p->shadow, ws, ws_bytes, w.frag.off, s);
        }
        const uint16_t *frag = reinterpret_cast<const uint16_t *>(wsp(ws, w.frag));
        FusedArgs a{};
        for (int net = 0; net < 2; ++net) {
            FusedNet &n = a.net[net];
            for (int l = 0; l < g.L; ++l) {
                n.W[l] = frag + w.frag_w[net][l];
                n.bias[l] = p->theta + (net == 0 ? g.ba[l] : g.bc[l]);
            }
            n.Wout = p->theta + (net == 0 ? g.Wa[g.L] : g.Wc[g.L]);
            n.bout = p->theta + (net == 0 ? g.ba[g.L] : g.bc[g.L]);
        }
        a.L = g.L;
        a.D = g.D;
        a.kpad = w.kpad;
        a.A = g.A;
        for (int l = 0; l < g.L; ++l) a.H[l] = g.H[l];
        a.obs = obs;
        a.B = N;
        a.M = N;
        a.logstd = p->theta + g.logstd;
        a.act_out = actions;
        a.logp_out = logp;
        a.val_out = values;
        a.mu_out = mu;
        a.key0 = static_cast<uint32_t>(seed);
        a.key1 = static_cast<uint32_t>(seed >> 32);
        a.t_step = static_cast<uint32_t>(t);
        a.iteration = iteration;
        a.net_mask = (value_only ? 0 : 1) | (values ? 2 : 0);
        a.vec_out = g.A % 4 == 0 && (!actions || aligned16(actions)) && (!mu || aligned16(mu)) ? 1 : 0;
        a.R = fsh.rows;
        a.NT = fsh.threads;
        PPO_HIP(launch_fused_infer(a, s), "fused inference");
        return PPO_OK;
    }
    note_ws_used(ws, ws_bytes);
    Tuning tune;
    PPO_CHECK(ensure_tuned(c, p, w, ws, N, false, s, tune));
    PPO_HIP(launch_stage_weights(c->prec, build_stage(c, p, w, ws, false), s), "stage_weights");
    PPO_HIP(launch_gather_obs(c->prec, s, obs, nullptr, N, N, g.D, w.kpad, wsp(ws, w.xg)), "gather_obs");
    PPO_HIP(enqueue_forward(c, p, w, ws, N, !value_only, values != nullptr, tune, s), "forward GEMM");
    HeadSampleArgs a{};
    a.ha = wsp(ws, w.h_a[g.L - 1]);
    a.hc = wsp(ws, w.h_c[g.L - 1]);
    a.Wa = p->theta + g.Wa[g.L];
    a.ba = p->theta + g.ba[g.L];
    a.logstd = p->theta + g.logstd;
    a.Wc = p->theta + g.Wc[g.L];
    a.bc = p->theta + g.bc[g.L];
    a.actions = actions;
    a.logp = logp;
    a.values = values;
    a.mu = mu;
    a.N = N;
    a.A = g.A;
    a.Hl = g.H[g.L - 1];
    a.key0 = static_cast<uint32_t>(seed);
    a.key1 = static_cast<uint32_t>(seed >> 32);
    a.t = static_cast<uint32_t>(t);
    a.iteration = iteration;
    a.value_only = value_only ? 1 : 0;
    PPO_HIP(launch_head_sample(c->prec, a, s), "head_sample");
    return PPO_OK;
}

namespace {

// Arguments shared by ppo_gae and ppo_gae_noalloc, checked before anything is
// enqueued.
int validate_gae(const ppo_ctx *c, const float *rewards, const uint8_t *dones, const uint8_t *timeouts,
                 const float *values, const float *last_values, int32_t T, int32_t N, float gamma, float lam,
                 const float *adv, const float *returns, const double *adv_stats, int32_t normalize) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    if (T < 1 || T > PPO_MAX_T) return fail(PPO_E_SHAPE, "T = %d outside 1..%d", T, PPO_MAX_T);
    if (N < 1) return fail(PPO_E_SHAPE, "N = %d must be positive", N);
    if (static_cast<long long>(T) * N < 2) return fail(PPO_E_SHAPE, "T * N must be at least 2");
    PPO_CHECK(check_ptr(rewards, "rewards"));
    PPO_CHECK(check_ptr(dones, "dones"));
    PPO_CHECK(check_ptr(timeouts, "timeouts", true));
    PPO_CHECK(check_ptr(values, "values"));
    PPO_CHECK(check_ptr(last_values, "last_values"));
    PPO_CHECK(check_ptr(adv, "adv"));
    PPO_CHECK(check_ptr(returns, "returns"));
    PPO_CHECK(check_ptr(adv_stats, "adv_stats"));
    if (!(gamma >= 0.0f && gamma <= 1.0f) || !(lam >= 0.0f && lam <= 1.0f))
        return fail(PPO_E_INVAL, "gamma and lambda must lie in [0, 1]");
    if (normalize != 0 && normalize != 1) return fail(PPO_E_INVAL, "normalize must be 0 or 1");
    return PPO_OK;
}

// The scan with its per-block statistics partials in `partials` (gae_blocks(N)
// x 3 doubles, every entry written before it is read), then the merge and the
// optional normalisation.
int enqueue_gae(hipStream_t s, const float *rewards, const uint8_t *dones, const uint8_t *timeouts,
                const float *values, const float *last_values, int32_t T, int32_t N, float gamma, float lam,
                float *adv, float *returns, double *adv_stats, int32_t normalize, double *partials) {
    GaeArgs a{};
    a.rewards = rewards;
    a.values = values;
    a.last_values = last_values;
    a.dones = dones;
    a.timeouts = timeouts;
    a.adv = adv;
    a.returns = returns;
    a.partials = partials;
    a.T = T;
    a.N = N;
    a.gamma = gamma;
    a.lam = lam;
    PPO_HIP(launch_gae(a, s), "gae");
    PPO_HIP(launch_adv_finalize(a.partials, gae_blocks(N), adv, static_cast<long long>(T) * N, adv_stats, normalize, s),
            "adv_finalize");
    return PPO_OK;
}

}  // namespace

int ppo_gae(const ppo_ctx *c, void *stream, const float *rewards, const uint8_t *dones, const uint8_t *timeouts,
            const float *values, const float *last_values, int32_t T, int32_t N, float gamma, float lam, float *adv,
            float *returns, double *adv_stats, int32_t normalize, void *ws, size_t ws_bytes) {
    PPO_CHECK(validate_gae(c, rewards, dones, timeouts, values, last_values, T, N, gamma, lam, adv, returns,
                           adv_stats, normalize));
    PPO_CHECK(validate_ws(c, N, T, 0, ws, ws_bytes));
    note_ws_used(ws, ws_bytes);
    PPO_CHECK(check_device());
    const WsPlan w = plan_workspace(c->g, c->prec, N, T, 0);
    return enqueue_gae(static_cast<hipStream_t>(stream), rewards, dones, timeouts, values, last_values, T, N, gamma,
                       lam, adv, returns, adv_stats, normalize, reinterpret_cast<double *>(wsp(ws, w.gae_part)));
}

static_assert(PPO_GAE_NOALLOC_MAX_N == kGaeNoAllocMaxN, "header limit and scratch size agree");

int ppo_gae_noalloc(const ppo_ctx *c, void *stream, const float *rewards, const uint8_t *dones,
                    const uint8_t *timeouts, const float *values, const float *last_values, int32_t T, int32_t N,
                    float gamma, float lam, float *adv, float *returns, double *adv_stats, int32_t normalize) {
    PPO_CHECK(validate_gae(c, rewards, dones, timeouts, values, last_values, T, N, gamma, lam, adv, returns,
                           adv_stats, normalize));
    if (N > PPO_GAE_NOALLOC_MAX_N)
        return fail(PPO_E_SHAPE, "N = %d exceeds PPO_GAE_NOALLOC_MAX_N = %d (the library's fixed scratch)", N,
                    PPO_GAE_NOALLOC_MAX_N);
    PPO_CHECK(check_device());
    double *partials = nullptr;
    PPO_HIP(gae_scratch(&partials), "scratch address");
    return enqueue_gae(static_cast<hipStream_t>(stream), rewards, dones, timeouts, values, last_values, T, N, gamma,
                       lam, adv, returns, adv_stats, normalize, partials);
}

int ppo_loss_grad(const ppo_ctx *c, void *stream, const ppo_params *p, const ppo_batch *b, const int32_t *idx,
                  int32_t M, const ppo_hparams *hp, float *stats, float *grad_out, uint8_t *active_out,
                  float *ratio_out, void *ws, size_t ws_bytes) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    PPO_CHECK(validate_hparams(hp));
    PPO_CHECK(validate_params(c, p, false));
    PPO_CHECK(validate_batch(c, b, hp));
    if (M < 1 || M > b->B) return fail(PPO_E_SHAPE, "M = %d outside 1..B", M);
    PPO_CHECK(check_ptr(idx, "idx"));
    PPO_CHECK(check_ptr(stats, "stats"));
    PPO_CHECK(check_ptr(grad_out, "grad_out", true));
    if (ratio_out && (reinterpret_cast<uintptr_t>(ratio_out) & 3u))
        return fail(PPO_E_INVAL, "ratio_out is not 4-byte aligned");
    PPO_CHECK(validate_ws(c, 0, 0, M, ws, ws_bytes));
    PPO_CHECK(check_device());
    note_ws_used(ws, ws_bytes);
    const WsPlan w = plan_workspace(c->g, c->prec, 0, 0, M);
    StepBuffers sb{b, idx, M, grad_out, stats, 0, 0};
    sb.active_out = active_out;
    sb.loss_only = grad_out == nullptr;
    sb.ratio_out = ratio_out;
    Tuning tune;
    PPO_CHECK(ensure_tuned(c, p, w, ws, M, true, static_cast<hipStream_t>(stream), tune, grad_out));
    PPO_HIP(enqueue_step(c, p, hp, w, ws, sb, tune, static_cast<hipStream_t>(stream)), "loss_grad");
    return PPO_OK;
}

int ppo_update_epoch(ppo_ctx *c, void *stream, const ppo_params *p, const ppo_batch *b, const int32_t *perm,
                     int32_t n_minibatches, const ppo_hparams *hp, float *stats, void *ws, size_t ws_bytes) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    PPO_CHECK(validate_hparams(hp));
    PPO_CHECK(validate_params(c, p, true));
    PPO_CHECK(validate_batch(c, b, hp));
    if (!perm) return fail(PPO_E_SHAPE, "perm is NULL");
    PPO_CHECK(check_ptr(perm, "perm"));
    if (n_minibatches < 1 || n_minibatches > b->B) return fail(PPO_E_SHAPE, "n_minibatches = %d", n_minibatches);
    if (b->B % n_minibatches != 0)
        return fail(PPO_E_SHAPE, "B = %d is not divisible by n_minibatches = %d", b->B, n_minibatches);
    PPO_CHECK(check_ptr(stats, "stats"));
    const int M = b->B / n_minibatches;
    PPO_CHECK(validate_ws(c, 0, 0, M, ws, ws_bytes));
    PPO_CHECK(check_device());

    const hipStream_t s = static_cast<hipStream_t>(stream);
    note_ws_used(ws, ws_bytes);
    note_shadow_written(p->shadow, s);
    const WsPlan w = plan_workspace(c->g, c->prec, 0, 0, M);
    Tuning tune;
    PPO_CHECK(ensure_tuned(c, p, w, ws, M, true, s, tune, p->grad));
    auto enqueue_all = [&](hipStream_t target) -> hipError_t {
        for (int k = 0; k < n_minibatches; ++k) {
            StepBuffers sb{b, perm + static_cast<long long>(k) * M, M, p->grad, stats + k * PPO_STATS_WIDTH, 1, k};
            // after the first step, Adam leaves the fragments of the next one in place
            sb.frags_ready = k > 0;
            sb.write_frags = k + 1 < n_minibatches;
            hipError_t e = enqueue_step(c, p, hp, w, ws, sb, tune, target);
            if (e != hipSuccess) return e;
        }
        return launch_step_advance(p->step, n_minibatches, target);
    };
    if (!hp->use_graph) {
        PPO_HIP(enqueue_all(s), "update_epoch");
        return PPO_OK;
    }

    std::lock_guard<std::mutex> lk(c->mu);
    PPO_CHECK(ensure_capture_stream(c));
    std::vector<uint64_t> key = {u64(p->theta), u64(p->grad), u64(p->adam_m), u64(p->adam_v), u64(p->shadow),
                                 u64(p->step), u64(p->lr), u64(b->obs), u64(b->actions), u64(b->logp),
                                 u64(b->adv), u64(b->returns), u64(b->values), u64(b->mu_old),
                                 u64(b->logstd_old), static_cast<uint64_t>(b->B),
                                 u64(perm), static_cast<uint64_t>(n_minibatches), u64(stats), u64(ws),
                                 fbits(hp->clip), fbits(hp->value_coef), fbits(hp->entropy_coef),
                                 fbits(hp->max_grad_norm), fbits(hp->beta1), fbits(hp->beta2), fbits(hp->adam_eps),
                                 static_cast<uint64_t>(hp->clip_value), fbits(hp->desired_kl),
                                 fbits(hp->lr_factor), fbits(hp->lr_min), fbits(hp->lr_max)};
    auto it = c->graphs.find(key);
    hipGraphExec_t exec = nullptr;
    if (it != c->graphs.end()) {
        exec = it->second;
    } else {
        PPO_HIP(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        hipError_t e = enqueue_all(c->capture);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->capture, &graph);
        if (e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(e, "capture of update_epoch");
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        if (c->graphs.size() >= kMaxGraphs) {
            auto old = c->graphs.find(c->graph_order.front());
            if (old != c->graphs.end()) {
                (void)hipGraphExecDestroy(old->second);
                c->graphs.erase(old);
            }
            c->graph_order.erase(c->graph_order.begin());
        }
        c->graphs[key] = exec;
        c->graph_order.push_back(key);
    }
    PPO_HIP(hipGraphLaunch(exec, s), "hipGraphLaunch");
    return PPO_OK;
}

int ppo_update_epoch_profiled(ppo_ctx *c, void *stream, const ppo_params *p, const ppo_batch *b,
                              const int32_t *perm, int32_t n_minibatches, const ppo_hparams *hp, float *stats,
                              void *ws, size_t ws_bytes, int32_t reps, float *phase_ms, int32_t *phase_launches) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    if (!phase_ms || !phase_launches) return fail(PPO_E_INVAL, "phase_ms and phase_launches are required");
    if (reps < 1 || reps > 1000) return fail(PPO_E_INVAL, "reps = %d outside 1..1000", reps);
    PPO_CHECK(validate_hparams(hp));
    PPO_CHECK(validate_params(c, p, true));
    PPO_CHECK(validate_batch(c, b, hp));
    if (!perm) return fail(PPO_E_SHAPE, "perm is NULL");
    PPO_CHECK(check_ptr(perm, "perm"));
    if (n_minibatches < 1 || n_minibatches > b->B) return fail(PPO_E_SHAPE, "n_minibatches = %d", n_minibatches);
    if (b->B % n_minibatches != 0)
        return fail(PPO_E_SHAPE, "B = %d is not divisible by n_minibatches = %d", b->B, n_minibatches);
    PPO_CHECK(check_ptr(stats, "stats"));
    const int M = b->B / n_minibatches;
    PPO_CHECK(validate_ws(c, 0, 0, M, ws, ws_bytes));
    PPO_CHECK(check_device());

    const hipStream_t s = static_cast<hipStream_t>(stream);
    note_ws_used(ws, ws_bytes);
    note_shadow_written(p->shadow, s);
    const WsPlan w = plan_workspace(c->g, c->prec, 0, 0, M);
    Tuning tune;
    PPO_CHECK(ensure_tuned(c, p, w, ws, M, true, s, tune, p->grad));
    Profiler prof;
    prof.s = s;
    prof.reps = reps;
    prof.reduce_repeatable = !(hp->desired_kl > 0.0f);
    for (int k = 0; k < n_minibatches; ++k) {
        StepBuffers sb{b, perm + static_cast<long long>(k) * M, M, p->grad, stats + k * PPO_STATS_WIDTH, 1, k};
        sb.frags_ready = k > 0;
        sb.write_frags = k + 1 < n_minibatches;
        PPO_HIP(enqueue_step(c, p, hp, w, ws, sb, tune, s, &prof), "update_epoch (profiled)");
    }
    PPO_HIP(launch_step_advance(p->step, n_minibatches, s), "step_advance");
    PPO_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int q = 0; q < PPO_N_PHASES; ++q) {
        phase_ms[q] = 0.0f;
        phase_launches[q] = 0;
    }
    for (size_t i = 0; i < prof.phase.size(); ++i) {
        float ms = 0.0f;
        PPO_HIP(hipEventElapsedTime(&ms, prof.ev[2 * i], prof.ev[2 * i + 1]), "hipEventElapsedTime");
        phase_ms[prof.phase[i]] += ms / prof.reps_for(prof.phase[i]);
        phase_launches[prof.phase[i]] += 1;
    }
    return PPO_OK;
}

int ppo_gemm_check(void *stream, int32_t precision, int32_t a_mode, int32_t b_mode, int32_t epilogue, int32_t M,
                   int32_t N, int32_t K, const void *A, int32_t lda, const void *B, int32_t ldb, void *C,
                   int32_t ldc, const float *bias, const void *H, int32_t ldh, float *rowsum, int32_t splits,
                   int32_t tile) {
    if (precision != PPO_FP32 && precision != PPO_BF16) return fail(PPO_E_INVAL, "precision %d", precision);
    if (tile < 0 || tile >= kNumTileShapes) return fail(PPO_E_INVAL, "tile %d", tile);
    const bool combo_ok = (a_mode == 0 && b_mode == 0 && epilogue == kEpiBiasElu) ||
                          (a_mode == 0 && b_mode == 0 && epilogue == kEpiDElu) ||
                          (a_mode == 0 && b_mode == 1 && epilogue == kEpiDElu) ||
                          (a_mode == 1 && b_mode == 1 && epilogue == kEpiPartial);
    if (!combo_ok) return fail(PPO_E_INVAL, "unsupported operand modes / epilogue combination");
    if (M < 1 || N < 1 || K < 1) return fail(PPO_E_SHAPE, "M, N, K must be positive");
    if (lda < (a_mode == 0 ? K : M) || ldb < (b_mode == 0 ? K : N) || ldc < N)
        return fail(PPO_E_SHAPE, "leading dimension too small");
    PPO_CHECK(check_ptr(A, "A"));
    PPO_CHECK(check_ptr(B, "B"));
    PPO_CHECK(check_ptr(C, "C"));
    if (epilogue == kEpiBiasElu) PPO_CHECK(check_ptr(bias, "bias"));
    if (epilogue == kEpiDElu) {
        PPO_CHECK(check_ptr(H, "H"));
        if (ldh < N) return fail(PPO_E_SHAPE, "ldh too small");
    }
    if (epilogue == kEpiPartial) PPO_CHECK(check_ptr(rowsum, "rowsum"));
    if (splits < 1 || (epilogue != kEpiPartial && splits != 1)) return fail(PPO_E_SHAPE, "splits = %d", splits);
    PPO_CHECK(check_device());
    const Precision prec = precision == PPO_BF16 ? kBF16 : kFP32;
    const int bk = gemm_bk(prec);
    GemmArgs args{};
    GemmProblem q{};
    q.A = A;
    q.B = B;
    q.C = C;
    q.bias = bias;
    q.H = H;
    q.rowsum = rowsum;
    q.M = M;
    q.N = N;
    q.K = K;
    q.lda = lda;
    q.ldb = ldb;
    q.ldc = ldc;
    q.ldh = ldh;
    q.c_split_stride = static_cast<long long>(M) * ldc;
    if (epilogue == kEpiPartial) {
        q.kps = cdiv(cdiv(K, splits), bk) * bk;
        q.splits = cdiv(K, q.kps);
    }
    args.tile = tile;
    add_problem(args, q, bk);
    PPO_HIP(launch_gemm(prec, a_mode, b_mode, epilogue, args, static_cast<hipStream_t>(stream)), "gemm");
    return PPO_OK;
}

}  // extern "C"

// ------------------------------------------------------ batched update
namespace {

// Appends every problem of `src` to `dst`, starting new launches when one
// fills up; all launches share `tile`.
void append_problems(std::vector<GemmArgs> &dst, const GemmArgs &src, int tile, int bk) {
    for (int i = 0; i < src.count; ++i) {
        if (dst.empty() || dst.back().count == kGemmMaxProblems) {
            dst.push_back(GemmArgs{});
            dst.back().tile = tile;
        }
        add_problem(dst.back(), src.p[i], bk);
    }
}

struct BatchedRun {
    const ppo_ctx *c;
    const ppo_params *p;
    const ppo_batch *b;
    const int32_t *perm;
    float *stats;
    void *ws;
    WsPlan w;
    int M;
};

// Tile choices of the grouped launches.  With autotuning off every site
// uses 128 x 128 tiles and each run keeps the weight-gradient split count it
// would use alone (results then equal each run's own ppo_update_epoch bit
// for bit); with autotuning on, the tiles are timed per grouped site and the
// weight-gradient workgroups of all runs get one common k-length, so the
// uneven runs finish their workgroups at about the same time.
struct BatchedTuning {
    int fwd[kMaxHidden] = {kTile128x128, kTile128x128, kTile128x128, kTile128x128};
    int dx[kMaxHidden] = {kTile128x128, kTile128x128, kTile128x128, kTile128x128};
    int dw = kTile128x128;
    int dw_kps[kMaxHidden + 1] = {0, 0, 0, 0, 0};   // per layer; 0: each run's own split count
};

// Per-layer common k-length: the weight-gradient problems of layer l of all
// runs share one launch, sized to `rounds` rounds of resident workgroups.
void batched_dw_kps(const std::vector<BatchedRun> &runs, int tile, int rounds, int *kps_out) {
    const int L = runs[0].c->g.L;
    const int bk = gemm_bk(runs[0].c->prec);
    for (int l = 0; l <= L; ++l) {
        long long work = 0;  // tile-samples
        for (const BatchedRun &r : runs)
            for (int net = 0; net < 2; ++net) {
                int rows, cols;
                dw_shape(r.c->g, net == 0, l, rows, cols);
                work += static_cast<long long>(cdiv(rows, tile_rows(tile))) * cdiv(cols, tile_cols(tile)) * r.M;
            }
        long long kps = (work + static_cast<long long>(rounds) * kResidentSlots - 1) / (rounds * kResidentSlots);
        kps = std::max<long long>(kps, 2 * bk);
        for (const BatchedRun &r : runs) {
            // never more splits than the workspace holds for that run
            const int min_kps = cdiv(cdiv(r.M, r.w.max_splits), bk) * bk;
            kps = std::max<long long>(kps, min_kps);
        }
        kps_out[l] = static_cast<int>(cdiv(kps, bk) * bk);
    }
}

// Weight-gradient launches of all runs, one group per layer (both networks
// of every run), so each launch holds like-sized work from every run.
std::vector<GemmArgs> batched_dw_launches(const std::vector<DwPlan> &plans, int L, int tile, int bk) {
    std::vector<GemmArgs> out;
    for (int l = 0; l <= L; ++l) {
        out.push_back(GemmArgs{});  // each layer starts a launch of its own
        out.back().tile = tile;
        for (const DwPlan &d : plans)
            for (int net = 0; net < 2; ++net) {
                const int i = net * (L + 1) + l;
                const GemmProblem &q = d.launch[i / kGemmMaxProblems].p[i % kGemmMaxProblems];
                if (out.back().count == kGemmMaxProblems) {
                    out.push_back(GemmArgs{});
                    out.back().tile = tile;
                }
                add_problem(out.back(), q, bk);
            }
    }
    return out;
}

// Side streams for the per-run kernels of a batched step: the runs' small
// launches (gather, loss, reduction, Adam) are independent of each other, so
// they fork from the caller's stream onto these streams and join back
// before the next grouped GEMM launch.  Captured into the epoch's graph they
// become parallel branches.  Default priority, library-owned, per device.
constexpr int kSideStreams = 4;
struct SideStreams {
    int dev = -1;
    hipStream_t st[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
};

int ensure_side_streams(SideStreams &ss, int dev) {
    if (ss.dev == dev) return PPO_OK;
    for (int i = 0; i < kSideStreams; ++i) {
        if (ss.st[i]) (void)hipStreamDestroy(ss.st[i]);
        if (ss.join[i]) (void)hipEventDestroy(ss.join[i]);
        ss.st[i] = nullptr;
        ss.join[i] = nullptr;
    }
    if (ss.fork) (void)hipEventDestroy(ss.fork);
    ss.fork = nullptr;
    ss.dev = -1;
    for (int i = 0; i < kSideStreams; ++i) {
        PPO_HIP(hipStreamCreateWithFlags(&ss.st[i], hipStreamNonBlocking), "hipStreamCreate (side)");
        PPO_HIP(hipEventCreateWithFlags(&ss.join[i], hipEventDisableTiming), "hipEventCreate");
    }
    PPO_HIP(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming), "hipEventCreate");
    ss.dev = dev;
    return PPO_OK;
}

hipError_t fork_to(const SideStreams &ss, hipStream_t s, int n) {
    hipError_t e = hipEventRecord(ss.fork, s);
    for (int i = 0; i < n && e == hipSuccess; ++i) e = hipStreamWaitEvent(ss.st[i], ss.fork, 0);
    return e;
}

hipError_t join_from(const SideStreams &ss, hipStream_t s, int n) {
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        e = hipEventRecord(ss.join[i], ss.st[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ss.join[i], 0);
    }
    return e;
}

// Step k of every run: per-run gathers, then one grouped launch per GEMM
// site covering all runs, per-run loss, reduce and Adam kernels (on side
// streams when given).
hipError_t enqueue_batched_step(std::vector<BatchedRun> &runs, const ppo_hparams *hp, int k,
                                const BatchedTuning &bt, hipStream_t s, const SideStreams *side) {
    const int R = static_cast<int>(runs.size());
    const NetLayout &g0 = runs[0].c->g;
    const Precision prec = runs[0].c->prec;
    const int bk = gemm_bk(prec);
    const int L = g0.L;
    const int n_side = side ? std::min(R, kSideStreams) : 0;
    auto run_stream = [&](int i) { return n_side > 0 ? side->st[i % n_side] : s; };
    hipError_t e;
    // every run through the fused per-sample pass when all of them can take
    // it: one pass per run on the side streams, concurrently, then the
    // grouped weight gradients; else the grouped layer-by-layer launches
    std::vector<FusedShape> fsh(R);
    bool all_fused = true;
    for (int i = 0; i < R; ++i) {
        fsh[i] = fused_shape_for(runs[i].c, runs[i].p, runs[i].w, runs[i].b->B);
        all_fused = all_fused && fsh[i].rows > 0;
    }
    if (n_side > 0 && (e = fork_to(*side, s, n_side)) != hipSuccess) return e;
    for (int i = 0; i < R; ++i) {
        BatchedRun &r = runs[i];
        const int32_t *idx = r.perm + static_cast<long long>(k) * r.M;
        if (all_fused) {
            e = launch_pack_frags(build_frags(r.c, r.p, r.w, r.ws), run_stream(i));
            if (e != hipSuccess) return e;
            FusedArgs fa = fused_args(r.c, r.p, hp, r.w, r.ws, r.b, idx, r.M);
            fa.R = fsh[i].rows;
            fa.NT = fsh[i].threads;
            fa.per_cu = fsh[i].per_cu;
            e = launch_fused_update(fa, run_stream(i));
            if (e != hipSuccess) return e;
            continue;
        }
        e = launch_stage_weights(prec, build_stage(r.c, r.p, r.w, r.ws, true), run_stream(i));
        if (e != hipSuccess) return e;
        e = launch_gather_obs(prec, run_stream(i), r.b->obs, idx, r.b->B, r.M, r.c->g.D, r.w.kpad,
                              wsp(r.ws, r.w.xg));
        if (e != hipSuccess) return e;
    }
    if (n_side > 0 && (e = join_from(*side, s, n_side)) != hipSuccess) return e;
    for (int l = 0; l < L && !all_fused; ++l) {
        std::vector<GemmArgs> launches;
        for (BatchedRun &r : runs)
            append_problems(launches, build_fwd(r.c, r.p, r.w, r.ws, r.M, l, true, true, bt.fwd[l]), bt.fwd[l], bk);
        for (const GemmArgs &a : launches) {
            e = launch_gemm(prec, 0, 0, kEpiBiasElu, a, s);
            if (e != hipSuccess) return e;
        }
    }
    if (!all_fused) {
        if (n_side > 0 && (e = fork_to(*side, s, n_side)) != hipSuccess) return e;
        for (int i = 0; i < R; ++i) {
            BatchedRun &r = runs[i];
            const HeadLossArgs hl = head_loss_args(r.c, r.p, hp, r.w, r.ws, r.b,
                                                   r.perm + static_cast<long long>(k) * r.M, r.M);
            e = launch_head_loss(prec, hl, run_stream(i));
            if (e != hipSuccess) return e;
        }
        if (n_side > 0 && (e = join_from(*side, s, n_side)) != hipSuccess) return e;
    }
    for (int l = L - 1; l >= 1 && !all_fused; --l) {
        std::vector<GemmArgs> launches;
        for (BatchedRun &r : runs)
            append_problems(launches, build_dx(r.c, r.p, r.w, r.ws, r.M, l, bt.dx[l]), bt.dx[l], bk);
        for (const GemmArgs &a : launches) {
            e = launch_gemm(prec, 0, 0, kEpiDElu, a, s);
            if (e != hipSuccess) return e;
        }
    }
    std::vector<DwPlan> plans(R);
    for (int i = 0; i < R; ++i) {
        TileChoice tc;
        tc.tile = bt.dw;
        tc.rounds = 2;
        plans[i] = build_dw(runs[i].c, runs[i].w, runs[i].ws, runs[i].M, tc, bt.dw_kps);
    }
    const std::vector<GemmArgs> launches = batched_dw_launches(plans, L, bt.dw, bk);
    for (const GemmArgs &a : launches) {
        e = launch_gemm(prec, 1, 1, kEpiPartial, a, s);
        if (e != hipSuccess) return e;
    }
    if (n_side > 0 && (e = fork_to(*side, s, n_side)) != hipSuccess) return e;
    for (int i = 0; i < R; ++i) {
        BatchedRun &r = runs[i];
        ReduceArgs &red = plans[i].red;
        set_reduce_loss(red, r.c, r.p, hp, r.w, r.ws, r.p->grad, r.M, 1, all_fused ? fsh[i].rows : 0);
        e = launch_grad_reduce(red, run_stream(i));
        if (e != hipSuccess) return e;
        const AdamArgs ad = adam_args(r.c, r.p, hp, red, r.p->grad, r.stats + k * PPO_STATS_WIDTH, r.M, k, 1);
        e = launch_adam(ad, run_stream(i));
        if (e != hipSuccess) return e;
    }
    if (n_side > 0 && (e = join_from(*side, s, n_side)) != hipSuccess) return e;
    return hipSuccess;
}

// Times one grouped GEMM site over all runs for a candidate.
template <typename Build>
hipError_t time_grouped(const std::vector<BatchedRun> &runs, int a_mode, int b_mode, int epi, int tile,
                        Build &&build, hipStream_t s, float &ms) {
    const int bk = gemm_bk(runs[0].c->prec);
    std::vector<GemmArgs> launches;
    for (const BatchedRun &r : runs) {
        std::vector<GemmArgs> one = build(r);
        for (const GemmArgs &a : one) append_problems(launches, a, tile, bk);
    }
    return time_launch(
        s,
        [&] {
            hipError_t e = hipSuccess;
            for (const GemmArgs &a : launches)
                if (e == hipSuccess) e = launch_gemm(runs[0].c->prec, a_mode, b_mode, epi, a, s);
            return e;
        },
        3, ms);
}

int tune_batched(std::vector<BatchedRun> &runs, hipStream_t s, BatchedTuning &bt) {
    bt = BatchedTuning{};
    if (!autotune_enabled()) return PPO_OK;
    const int L = runs[0].c->g.L;
    for (int l = 0; l < L; ++l) {
        float best = 1e30f;
        for (int tile = 0; tile < kNumTileShapes; ++tile) {
            float ms = 0.0f;
            PPO_HIP(time_grouped(runs, 0, 0, kEpiBiasElu, tile,
                                 [&](const BatchedRun &r) {
                                     return std::vector<GemmArgs>{
                                         build_fwd(r.c, r.p, r.w, r.ws, r.M, l, true, true, tile)};
                                 },
                                 s, ms),
                    "autotune grouped forward");
            if (ms < best) {
                best = ms;
                bt.fwd[l] = tile;
            }
        }
    }
    for (int l = 1; l < L; ++l) {
        float best = 1e30f;
        for (int tile = 0; tile < kNumTileShapes; ++tile) {
            float ms = 0.0f;
            PPO_HIP(time_grouped(runs, 0, 0, kEpiDElu, tile,
                                 [&](const BatchedRun &r) {
                                     return std::vector<GemmArgs>{build_dx(r.c, r.p, r.w, r.ws, r.M, l, tile)};
                                 },
                                 s, ms),
                    "autotune grouped input gradient");
            if (ms < best) {
                best = ms;
                bt.dx[l] = tile;
            }
        }
    }
    float best = 1e30f;
    const Precision prec = runs[0].c->prec;
    const int bk = gemm_bk(prec);
    for (int tile = 0; tile < kNumTileShapes; ++tile)
        for (int rounds : {1, 2, 4}) {
            int kps[kMaxHidden + 1] = {0, 0, 0, 0, 0};
            batched_dw_kps(runs, tile, rounds, kps);
            std::vector<DwPlan> plans;
            for (const BatchedRun &r : runs) {
                TileChoice tc;
                tc.tile = tile;
                plans.push_back(build_dw(r.c, r.w, r.ws, r.M, tc, kps));
            }
            const std::vector<GemmArgs> launches = batched_dw_launches(plans, L, tile, bk);
            float ms = 0.0f;
            PPO_HIP(time_launch(
                        s,
                        [&] {
                            hipError_t e = hipSuccess;
                            for (const GemmArgs &a : launches)
                                if (e == hipSuccess) e = launch_gemm(prec, 1, 1, kEpiPartial, a, s);
                            return e;
                        },
                        3, ms),
                    "autotune grouped weight gradient");
            if (ms < best) {
                best = ms;
                bt.dw = tile;
                for (int l = 0; l <= L; ++l) bt.dw_kps[l] = kps[l];
            }
        }
    return PPO_OK;
}

std::mutex g_batched_mu;
std::map<std::string, BatchedTuning> g_batched_tuning;
std::map<std::vector<uint64_t>, hipGraphExec_t> g_batched_graphs;
std::vector<std::vector<uint64_t>> g_batched_order;
hipStream_t g_batched_capture = nullptr;
int g_batched_dev = -1;
SideStreams g_side;

}  // namespace

extern "C" {

int ppo_update_batched(ppo_ctx *const *ctxs, int32_t R, void *stream, const ppo_params *params,
                       const ppo_batch *batches, const int32_t *const *perms, int32_t n_minibatches,
                       const ppo_hparams *hp, float *const *stats, void *const *ws, const size_t *ws_bytes) {
    if (!ctxs || !params || !batches || !perms || !stats || !ws || !ws_bytes)
        return fail(PPO_E_INVAL, "NULL array argument");
    if (R < 1 || R > PPO_MAX_RUNS) return fail(PPO_E_SHAPE, "R = %d outside 1..%d", R, PPO_MAX_RUNS);
    PPO_CHECK(validate_hparams(hp));
    std::vector<BatchedRun> runs(R);
    for (int i = 0; i < R; ++i) {
        const ppo_ctx *c = ctxs[i];
        if (!c) return fail(PPO_E_INVAL, "ctxs[%d] is NULL", i);
        if (c->prec != ctxs[0]->prec) return fail(PPO_E_INVAL, "runs differ in precision");
        if (c->g.L != ctxs[0]->g.L) return fail(PPO_E_SHAPE, "runs differ in the number of hidden layers");
        PPO_CHECK(validate_params(c, &params[i], true));
        PPO_CHECK(validate_batch(c, &batches[i], hp));
        if (!perms[i]) return fail(PPO_E_SHAPE, "perms[%d] is NULL", i);
        PPO_CHECK(check_ptr(perms[i], "perm"));
        if (n_minibatches < 1 || n_minibatches > batches[i].B || batches[i].B % n_minibatches != 0)
            return fail(PPO_E_SHAPE, "run %d: B = %d is not divisible by n_minibatches = %d", i, batches[i].B,
                        n_minibatches);
        PPO_CHECK(check_ptr(stats[i], "stats"));
        const int M = batches[i].B / n_minibatches;
        PPO_CHECK(validate_ws(c, 0, 0, M, ws[i], ws_bytes[i]));
        runs[i] = BatchedRun{c, &params[i], &batches[i], perms[i], stats[i], ws[i],
                             plan_workspace(c->g, c->prec, 0, 0, M), M};
    }
    PPO_CHECK(check_device());
    const hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < R; ++i) {
        note_ws_used(ws[i], ws_bytes[i]);
        note_shadow_written(params[i].shadow, s);
    }
    // When every run takes the fused pass, each run's whole epoch (its own
    // tuned steps, as ppo_update_epoch enqueues them) goes to one of the side
    // streams, the runs spread over them by work (largest first onto the
    // least loaded stream), with one fork and one join: the runs proceed
    // independently and the small ones fill the slots the large ones leave
    // free.  Otherwise step k of every run is enqueued together (grouped
    // GEMM launches across runs).  PPO_BATCHED_GROUPED=1 forces the latter.
    bool per_run = R > 1;
    if (const char *v = std::getenv("PPO_BATCHED_GROUPED")) per_run = per_run && std::strcmp(v, "1") != 0;
    for (int i = 0; i < R && per_run; ++i)
        per_run = fused_shape_for(runs[i].c, runs[i].p, runs[i].w, runs[i].b->B).rows > 0;
    BatchedTuning bt;
    std::vector<Tuning> tunes(R);
    std::vector<int> order(R), lane(R, 0);
    if (per_run) {
        std::vector<double> work(R);
        for (int i = 0; i < R; ++i) {
            PPO_CHECK(ensure_tuned(runs[i].c, runs[i].p, runs[i].w, runs[i].ws, runs[i].M, true, s, tunes[i],
                                   runs[i].p->grad));
            const NetLayout &g = runs[i].c->g;
            double per_sample = static_cast<double>(g.D) * g.H[0];
            for (int l = 1; l < g.L; ++l) per_sample += static_cast<double>(g.H[l - 1]) * g.H[l];
            work[i] = per_sample * runs[i].b->B;
            order[i] = i;
        }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
        double load[kSideStreams] = {};
        const int n_side = std::min(R, kSideStreams);
        for (int i : order) {
            int j = 0;
            for (int q = 1; q < n_side; ++q)
                if (load[q] < load[j]) j = q;
            lane[i] = j;
            load[j] += work[i];
        }
    } else {
        std::string key = std::string(autotune_enabled() ? "t" : "f");
        for (const BatchedRun &r : runs) key += "|" + tune_key(r.c, r.M, true);
        std::lock_guard<std::mutex> lk(g_batched_mu);
        auto it = g_batched_tuning.find(key);
        if (it != g_batched_tuning.end()) {
            bt = it->second;
        } else {
            PPO_CHECK(tune_batched(runs, s, bt));
            g_batched_tuning[key] = bt;
        }
    }
    auto enqueue_all = [&](hipStream_t target) -> hipError_t {
        hipError_t e;
        if (per_run) {
            const int n_side = std::min(R, kSideStreams);
            if ((e = fork_to(g_side, target, n_side)) != hipSuccess) return e;
            for (int i : order) {
                const BatchedRun &r = runs[i];
                const hipStream_t st = g_side.st[lane[i]];
                for (int k = 0; k < n_minibatches; ++k) {
                    StepBuffers sb{r.b, r.perm + static_cast<long long>(k) * r.M, r.M, r.p->grad,
                                   r.stats + k * PPO_STATS_WIDTH, 1, k};
                    sb.frags_ready = k > 0;
                    sb.write_frags = k + 1 < n_minibatches;
                    if ((e = enqueue_step(r.c, r.p, hp, r.w, r.ws, sb, tunes[i], st)) != hipSuccess) return e;
                }
                if ((e = launch_step_advance(r.p->step, n_minibatches, st)) != hipSuccess) return e;
            }
            return join_from(g_side, target, n_side);
        }
        for (int k = 0; k < n_minibatches; ++k) {
            e = enqueue_batched_step(runs, hp, k, bt, target, R > 1 ? &g_side : nullptr);
            if (e != hipSuccess) return e;
        }
        for (int i = 0; i < R; ++i) {
            e = launch_step_advance(params[i].step, n_minibatches, target);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    std::lock_guard<std::mutex> lk(g_batched_mu);
    int dev = 0;
    PPO_HIP(hipGetDevice(&dev), "hipGetDevice");
    PPO_CHECK(ensure_side_streams(g_side, dev));
    if (!hp->use_graph) {
        PPO_HIP(enqueue_all(s), "update_batched");
        return PPO_OK;
    }
    std::vector<uint64_t> key = {static_cast<uint64_t>(R), static_cast<uint64_t>(n_minibatches),
                                 fbits(hp->clip), fbits(hp->value_coef), fbits(hp->entropy_coef),
                                 fbits(hp->max_grad_norm), fbits(hp->beta1), fbits(hp->beta2), fbits(hp->adam_eps),
                                 static_cast<uint64_t>(hp->clip_value), fbits(hp->desired_kl),
                                 fbits(hp->lr_factor), fbits(hp->lr_min), fbits(hp->lr_max)};
    for (int i = 0; i < R; ++i) {
        const ppo_params &p = params[i];
        const ppo_batch &b = batches[i];
        for (uint64_t v : {u64(ctxs[i]), u64(p.theta), u64(p.grad), u64(p.adam_m), u64(p.adam_v), u64(p.shadow),
                           u64(p.step), u64(p.lr), u64(b.obs), u64(b.actions), u64(b.logp), u64(b.adv),
                           u64(b.returns), u64(b.values), u64(b.mu_old), u64(b.logstd_old),
                           static_cast<uint64_t>(b.B), u64(perms[i]), u64(stats[i]),
                           u64(ws[i])})
            key.push_back(v);
    }
    if (g_batched_capture && g_batched_dev != dev) {
        for (auto &kv : g_batched_graphs) (void)hipGraphExecDestroy(kv.second);
        g_batched_graphs.clear();
        g_batched_order.clear();
        (void)hipStreamDestroy(g_batched_capture);
        g_batched_capture = nullptr;
    }
    if (!g_batched_capture) {
        PPO_HIP(hipStreamCreateWithFlags(&g_batched_capture, hipStreamNonBlocking), "hipStreamCreate");
        g_batched_dev = dev;
    }
    hipGraphExec_t exec = nullptr;
    auto it = g_batched_graphs.find(key);
    if (it != g_batched_graphs.end()) {
        exec = it->second;
    } else {
        PPO_HIP(hipStreamBeginCapture(g_batched_capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        hipError_t e = enqueue_all(g_batched_capture);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(g_batched_capture, &graph);
        if (e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(e, "capture of update_batched");
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        if (g_batched_graphs.size() >= kMaxGraphs) {
            auto old = g_batched_graphs.find(g_batched_order.front());
            if (old != g_batched_graphs.end()) {
                (void)hipGraphExecDestroy(old->second);
                g_batched_graphs.erase(old);
            }
            g_batched_order.erase(g_batched_order.begin());
        }
        g_batched_graphs[key] = exec;
        g_batched_order.push_back(key);
    }
    PPO_HIP(hipGraphLaunch(exec, s), "hipGraphLaunch");
    return PPO_OK;
}

int ppo_ctx_tuning(const ppo_ctx *c, int32_t rows, int32_t update, int32_t *choices, int32_t capacity) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    if (!choices) return fail(PPO_E_INVAL, "choices is NULL");
    if (capacity < 2 * kNumSites) return fail(PPO_E_SHAPE, "capacity %d < %d", capacity, 2 * kNumSites);
    ppo_ctx *cc = const_cast<ppo_ctx *>(c);
    std::lock_guard<std::mutex> lk(cc->mu);
    auto it = cc->tuned.find(update ? -rows : rows);
    if (it == cc->tuned.end()) return fail(PPO_E_SHAPE, "no tile choice recorded for %d rows", rows);
    for (int i = 0; i < kNumSites; ++i) {
        choices[2 * i] = it->second.site[i].tile;
        choices[2 * i + 1] = it->second.site[i].rounds;
    }
    return PPO_OK;
}

}  // extern "C"

namespace {
int fused_shape_query(const ppo_ctx *c, int32_t *rows, int32_t *threads, bool inference) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    if (!rows || !threads) return fail(PPO_E_INVAL, "rows or threads is NULL");
    *rows = 0;
    *threads = 0;
    if (c->prec != kBF16 || !fused_env_enabled()) return PPO_OK;
    const WsPlan w = plan_workspace(c->g, c->prec, 0, 0, 1);
    const char *r = std::getenv("PPO_FUSED_ROWS");
    const char *t = std::getenv("PPO_FUSED_THREADS");
    const char *pc = inference ? nullptr : std::getenv("PPO_FUSED_PER_CU");
    FusedShape sh = fused_shape(c->g.L, c->g.H, w.kpad, c->g.A, r ? std::atoi(r) : 0, t ? std::atoi(t) : 0,
                                !inference, pc ? std::atoi(pc) : 0);
    *rows = sh.rows;
    *threads = sh.threads;
    return PPO_OK;
}

}  // namespace

extern "C" {

int ppo_fused_shape(const ppo_ctx *c, int32_t *rows, int32_t *threads) {
    return fused_shape_query(c, rows, threads, false);
}

int ppo_fused_infer_shape(const ppo_ctx *c, int32_t *rows, int32_t *threads) {
    return fused_shape_query(c, rows, threads, true);
}

int ppo_assemble_obs(const ppo_ctx *c, void *stream, const float *proprio, int32_t n_proprio, const float *base,
                     const ppo_terrain *terrain, const float *noise_scale, int32_t N, int32_t t, uint64_t seed,
                     uint32_t iteration, float *obs) {
    if (!c) return fail(PPO_E_INVAL, "ctx is NULL");
    const int D = c->net.obs_dim;
    const int S = terrain ? terrain->n_scan : 0;
    if (n_proprio < 0 || S < 0 || static_cast<long long>(n_proprio) + S != D)
        return fail(PPO_E_SHAPE, "n_proprio %d + n_scan %d must equal obs_dim %d", n_proprio, S, D);
    const long long groups = (D + 3) / 4;
    const long long n_max = std::min(1LL << 24, 0x7FFFFFFFLL / groups);
    if (N < 1 || N > n_max) return fail(PPO_E_SHAPE, "N = %d outside 1..%lld", N, n_max);
    if (t < 0) return fail(PPO_E_SHAPE, "t = %d must be non-negative", t);
    PPO_CHECK(check_ptr(proprio, "proprio", n_proprio == 0));
    PPO_CHECK(check_ptr(noise_scale, "noise_scale", true));
    PPO_CHECK(check_ptr(obs, "obs"));
    if (S > 0) {
        PPO_CHECK(check_ptr(base, "base"));
        PPO_CHECK(check_ptr(terrain->height, "terrain.height"));
        PPO_CHECK(check_ptr(terrain->scan, "terrain.scan"));
        if (terrain->nx < 1 || terrain->ny < 1 || terrain->nx > (1 << 24) || terrain->ny > (1 << 24))
            return fail(PPO_E_SHAPE, "height field %d x %d outside 1..2^24 per side", terrain->nx, terrain->ny);
        if (!(terrain->inv_res > 0.0f) || !std::isfinite(terrain->inv_res))
            return fail(PPO_E_INVAL, "terrain.inv_res must be positive and finite");
    }
    PPO_CHECK(check_device());
    PPO_HIP(launch_assemble_obs(static_cast<hipStream_t>(stream), proprio, n_proprio, base,
                                S > 0 ? terrain->height : nullptr, S > 0 ? terrain->nx : 1, S > 0 ? terrain->ny : 1,
                                S > 0 ? terrain->inv_res : 1.0f, S > 0 ? terrain->scan : nullptr, S, noise_scale, N, seed,
                                static_cast<uint32_t>(t), iteration, obs),
            "assemble_obs");
    return PPO_OK;
}

int ppo_philox_blocks(void *stream, uint64_t seed, uint32_t c0_base, uint32_t c1, uint32_t c2, uint32_t c3,
                      int64_t n, uint32_t *out) {
    if (n < 1 || n > (static_cast<int64_t>(1) << 28)) return fail(PPO_E_SHAPE, "n = %lld outside 1..2^28", (long long)n);
    PPO_CHECK(check_ptr(out, "out"));
    PPO_CHECK(check_device());
    PPO_HIP(launch_philox_blocks(static_cast<hipStream_t>(stream), seed, c0_base, c1, c2, c3, n, out), "philox");
    return PPO_OK;
}

}  // extern "C"
