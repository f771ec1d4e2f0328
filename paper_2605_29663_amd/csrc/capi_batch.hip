// C ABI of the batched multi-scene step (declared in include/exact_mppi.h):
// planning of the longest-first work queue, workspaces, eager execution,
// hipGraph capture and replay, and the tile autotuner of the batch.
#include "ctx.hpp"

using namespace emppi;
using namespace emppi_host;

struct mppi_batch_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int n = 0;
    std::vector<mppi_ctx> scenes;
    std::vector<mppi_params> prms;
    std::vector<StepArgs> args;     // static part of each scene's step arguments
    std::vector<int> u_off;         // offsets of the scenes' nominals in the packed array
    std::vector<uint64_t> noise_stream;  // Philox stream word of each scene (0 by default)
    // snapshot of what the plan was built from
    std::vector<int> snap_n;
    std::vector<const void*> snap_ptr;
    // plan
    double work_target = 0.0;       // requested pairs per queue item (0: default)
    double work_per_item = 0.0;     // point-primitive pairs per queue item of the plan
    int resident[2][DMIN_CLASSES] = {};  // resident workgroups of each persistent launch
    std::vector<SceneBufs> bufs;
    std::vector<SceneDmin> sdm;     // [pass][scene]
    std::vector<DminItem> items[2][DMIN_CLASSES];  // [pass][register class]
    std::vector<int2> blk_roll, blk_upd;
    DevBuf arena, d_steps, d_bufs, d_sdm, d_items[2][DMIN_CLASSES], d_blk_roll, d_blk_upd, d_counters, d_out;
    SceneStep* h_steps = nullptr;   // pinned
    float* h_out = nullptr;         // pinned
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool planned = false;
    bool stepped = false;           // a step ran since the workspaces were carved
    bool capturing = false;
    std::vector<int> cls_order[2];  // classes with items, most work first
    // HIP-event timing of the sampled-rollout signed-distance pass (eager steps)
    bool prof = false, prof_pending = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double prof_ms = 0.0;
    long long prof_n = 0;
};

static_assert(HYB_MAX_MODES == MPPI_MAX_MODES, "mode capacity of the C ABI");

struct mppi_hybrid_s {
    mppi_batch b = nullptr;
    int n = 0;
    int model[HYB_MAX_MODES] = {};
    int nu[HYB_MAX_MODES] = {};
    DevBuf d_res;
    float* h_res = nullptr;  // pinned
    std::string err;
};

namespace {

int bfail(mppi_batch b, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b)
        b->err = buf;
    else
        g_create_error = buf;
    return code;
}

#define BHIP(b, expr)                                                                         \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess)                                                                 \
            return bfail((b), MPPI_E_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));     \
    } while (0)

void drop_graph(mppi_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// The scene data the plan depends on: point count and buffer addresses.
void snapshot(mppi_batch b) {
    b->snap_n.clear();
    b->snap_ptr.clear();
    for (mppi_ctx c : b->scenes) {
        b->snap_n.push_back(c->n_points);
        b->snap_n.push_back(c->moving ? 1 : 0);
        b->snap_n.push_back(c->BP * 100 + c->RP);
        b->snap_ptr.push_back(c->px.p);
        b->snap_ptr.push_back(c->pvx.p);
        b->snap_ptr.push_back(c->poly_verts.p);
        b->snap_ptr.push_back(c->rects.p);
    }
}

bool snapshot_matches(mppi_batch b) {
    size_t k = 0, m = 0;
    for (mppi_ctx c : b->scenes) {
        if (b->snap_n[k++] != c->n_points || b->snap_n[k++] != (c->moving ? 1 : 0) ||
            b->snap_n[k++] != c->BP * 100 + c->RP)
            return false;
        if (b->snap_ptr[m++] != c->px.p || b->snap_ptr[m++] != c->pvx.p ||
            b->snap_ptr[m++] != c->poly_verts.p || b->snap_ptr[m++] != c->rects.p)
            return false;
    }
    return true;
}

// Build the work queue for a given target work per item, size and carve the
// workspace arena, and upload the static tables.
constexpr double DEFAULT_WORK_PER_ITEM = 4194304.0;
constexpr int TAIL_SPLIT_MIN_POINTS = 32;  // tail items are split while parts keep this many points
constexpr double MIN_WORK_PER_ITEM = 65536.0;

// Plan for queue items of `work_target` point-primitive pairs (0: the
// default, shrunk for small batches).
int plan(mppi_batch b, double work_target) {
    drop_graph(b);
    const int n = b->n;
    b->work_target = work_target;
    b->bufs.assign(n, SceneBufs{});
    b->sdm.assign(2 * n, SceneDmin{});
    for (auto& p : b->items)
        for (auto& v : p) v.clear();
    b->blk_roll.clear();
    b->blk_upd.clear();
    int cus = 0;
    BHIP(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    for (int pass = 0; pass < 2; ++pass)
        for (int cls = 0; cls < DMIN_CLASSES; ++cls) {
            const int per_cu = dmin_persistent_blocks_per_cu(cls, pass == 0 ? 256 : 128);
            if (per_cu <= 0 || cus <= 0)
                return bfail(b, MPPI_E_HIP, "occupancy query failed for the persistent kernel");
            b->resident[pass][cls] = cus * per_cu;
        }
    struct Cost {
        double c;
        DminItem it;
    };
    std::vector<Cost> q[2][DMIN_CLASSES];
    // arena layout
    std::vector<size_t> off(n * 9);
    size_t total = 0;
    std::vector<int> nchunk(n), chunk(n), nchunk_nom(n), chunk_nom(n);
    // default items: large for large batches (LPT balance needs few, big
    // items), shrunk for small batches so that the sampled-rollout pass
    // still has about two rounds of resident workgroups
    double total_pairs = 0.0;
    int slots = 1, val_slots = 1;  // resident workgroups of the classes this batch uses
    for (int s = 0; s < n; ++s) {
        const mppi_params& P = b->prms[s];
        mppi_ctx c = b->scenes[s];
        const int padded = P.footprint_kind == 0 ? c->BP : c->RP;
        total_pairs += static_cast<double>(b->args[s].Kpad) * P.T * std::max(c->n_points, 0) * padded;
        const int cls = dmin_class(P.footprint_kind, padded);
        slots = std::max(slots, b->resident[0][cls]);
        val_slots = std::max(val_slots, b->resident[1][cls]);
    }
    const double work_per_item =
        work_target > 0.0 ? std::max(MIN_WORK_PER_ITEM, work_target)
                          : std::max(MIN_WORK_PER_ITEM,
                                     std::min(DEFAULT_WORK_PER_ITEM, total_pairs / (2.0 * slots)));
    b->work_per_item = work_per_item;
    // validation pass (T poses per scene, one 128-lane tile): split each
    // scene's points so that all scenes together give about two rounds of
    // resident workgroups (chunks of at least 16 points)
    const int val_chunks = std::max(1, 2 * val_slots / std::max(n, 1));
    for (int s = 0; s < n; ++s) {
        const mppi_params& P = b->prms[s];
        mppi_ctx c = b->scenes[s];
        const int kind = P.footprint_kind;
        const int padded = kind == 0 ? c->BP : c->RP;
        const size_t Kpad = b->args[s].Kpad, T = P.T, nu = P.nu;
        const int npts = std::max(c->n_points, 0);
        // rollout pass: pose tiles of 256 lanes (fewer poses where a lane
        // group shares a pose), chunks sized for the target work
        const double per_point = 256.0 / dmin_persistent_lanes_per_pose(dmin_class(kind, padded)) * padded;
        int ck = static_cast<int>(std::max(32.0, std::min(static_cast<double>(std::max(npts, 1)),
                                                          work_per_item / per_point)));
        nchunk[s] = std::max(1, (npts + ck - 1) / ck);
        chunk[s] = std::max(1, (npts + nchunk[s] - 1) / nchunk[s]);
        // validation pass: the T poses in tiles of 128 lanes, small chunks
        const int ckn = std::max(16, (npts + val_chunks - 1) / val_chunks);
        nchunk_nom[s] = std::max(1, (npts + ckn - 1) / ckn);
        chunk_nom[s] = std::max(1, (npts + nchunk_nom[s] - 1) / nchunk_nom[s]);
        const size_t sizes[9] = {sizeof(float) * T * nu * Kpad, sizeof(float4) * T * Kpad,
                                 sizeof(float) * Kpad, sizeof(float) * Kpad,
                                 sizeof(unsigned int) * T * Kpad, sizeof(float) * T * nu,
                                 sizeof(float4) * T, sizeof(unsigned int) * T, 0};
        for (int k = 0; k < 9; ++k) {
            off[s * 9 + k] = total;
            total += align256(sizes[k]);
        }
    }
    BHIP(b, b->arena.ensure(std::max<size_t>(total, 256)));
    BHIP(b, b->d_out.ensure(sizeof(float) * OUT_FLOATS * n));
    char* base = static_cast<char*>(b->arena.p);
    for (int s = 0; s < n; ++s) {
        const mppi_params& P = b->prms[s];
        mppi_ctx c = b->scenes[s];
        const int kind = P.footprint_kind;
        const int padded = kind == 0 ? c->BP : c->RP;
        const int Kpad = b->args[s].Kpad, T = P.T;
        SceneBufs& B = b->bufs[s];
        B.eps_ws = reinterpret_cast<float*>(base + off[s * 9 + 0]);
        B.poses = reinterpret_cast<float4*>(base + off[s * 9 + 1]);
        B.jbase = reinterpret_cast<float*>(base + off[s * 9 + 2]);
        B.jt = reinterpret_cast<float*>(base + off[s * 9 + 3]);
        B.key = reinterpret_cast<unsigned int*>(base + off[s * 9 + 4]);
        B.unew = reinterpret_cast<float*>(base + off[s * 9 + 5]);
        B.nom = reinterpret_cast<float4*>(base + off[s * 9 + 6]);
        B.key_nom = reinterpret_cast<unsigned int*>(base + off[s * 9 + 7]);
        B.out = b->d_out.as<float>() + OUT_FLOATS * s;
        B.validate = P.validate ? 1 : 0;
        const int cls = dmin_class(kind, padded);
        for (int pass = 0; pass < 2; ++pass) {
            SceneDmin& D = b->sdm[pass * n + s];
            D.poses = pass == 0 ? B.poses : B.nom;
            D.npose = pass == 0 ? T * Kpad : T;
            D.pt = pass == 0 ? PoseTime{Kpad, T, b->args[s].state_offset, P.dt}
                             : PoseTime{1, T, b->args[s].state_offset, P.dt};
            D.pts = point_args(c);
            D.chunk = pass == 0 ? chunk[s] : chunk_nom[s];
            D.kind = kind;
            D.padded = padded;
            D.verts = c->poly_verts.as<float2>();
            D.rects = c->rects.as<float4>();
            D.key = pass == 0 ? B.key : B.key_nom;
            if (pass == 1 && !P.validate) continue;
            const int tile = (pass == 0 ? 256 : 128) / dmin_persistent_lanes_per_pose(cls);
            const int nck = pass == 0 ? nchunk[s] : nchunk_nom[s];
            for (int g0 = 0; g0 < D.npose; g0 += tile) {
                const int live = std::min(tile, D.npose - g0);
                for (int k = 0; k < nck; ++k) {
                    const int c0 = k * D.chunk;
                    const int len = std::max(0, std::min(D.chunk, c->n_points - c0));
                    q[pass][cls].push_back({static_cast<double>(live) * (len + 8) * padded,
                                            DminItem{pass * n + s, g0, c0, c0 + len}});
                }
            }
        }
        for (int r0 = 0; r0 < Kpad; r0 += WAVE) b->blk_roll.push_back(make_int2(s, r0));
        for (int h = 0; h < T; ++h) b->blk_upd.push_back(make_int2(s, h));
    }
    double class_work[2][DMIN_CLASSES] = {};
    for (int pass = 0; pass < 2; ++pass)
        for (int cls = 0; cls < DMIN_CLASSES; ++cls) {
            auto& v = q[pass][cls];
            std::stable_sort(v.begin(), v.end(), [](const Cost& x, const Cost& y) { return x.c > y.c; });
            // guided tail: the items of the last round of resident workgroups
            // (the smallest, after the longest-first sort) are split in four
            // along their point range, so the queue ends with quarter items
            // and the workgroups finish within a quarter item of each other
            double total = 0.0;
            for (const auto& e : v) total += e.c;
            const double round_work = v.empty() ? 0.0 : total / v.size() * b->resident[pass][cls];
            size_t cut = v.size();
            double suffix = 0.0;
            while (cut > 0 && suffix + v[cut - 1].c <= round_work) suffix += v[--cut].c;
            if (!v.empty()) class_work[pass][cls] = total;
            for (size_t i = 0; i < v.size(); ++i) {
                const DminItem it = v[i].it;
                const int len = it.c1 - it.c0;
                if (i < cut || len < 4 * TAIL_SPLIT_MIN_POINTS) {
                    b->items[pass][cls].push_back(it);
                    continue;
                }
                for (int part = 0; part < 4; ++part)
                    b->items[pass][cls].push_back(DminItem{it.sd, it.g0, it.c0 + part * len / 4,
                                                           it.c0 + (part + 1) * len / 4});
            }
        }
    for (int pass = 0; pass < 2; ++pass) {
        auto& o = b->cls_order[pass];
        o.clear();
        for (int cls = 0; cls < DMIN_CLASSES; ++cls)
            if (!b->items[pass][cls].empty()) o.push_back(cls);
        std::stable_sort(o.begin(), o.end(), [&](int x, int y) {
            return class_work[pass][x] > class_work[pass][y];
        });
    }
    // upload tables
    BHIP(b, hipStreamSynchronize(b->stream));
    BHIP(b, b->d_bufs.ensure(sizeof(SceneBufs) * n));
    BHIP(b, b->d_sdm.ensure(sizeof(SceneDmin) * 2 * n));
    BHIP(b, b->d_blk_roll.ensure(sizeof(int2) * std::max<size_t>(1, b->blk_roll.size())));
    BHIP(b, b->d_blk_upd.ensure(sizeof(int2) * std::max<size_t>(1, b->blk_upd.size())));
    BHIP(b, hipMemcpy(b->d_bufs.p, b->bufs.data(), sizeof(SceneBufs) * n, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_sdm.p, b->sdm.data(), sizeof(SceneDmin) * 2 * n, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_blk_roll.p, b->blk_roll.data(), sizeof(int2) * b->blk_roll.size(),
                      hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_blk_upd.p, b->blk_upd.data(), sizeof(int2) * b->blk_upd.size(),
                      hipMemcpyHostToDevice));
    for (int pass = 0; pass < 2; ++pass)
        for (int cls = 0; cls < DMIN_CLASSES; ++cls) {
            auto& v = b->items[pass][cls];
            BHIP(b, b->d_items[pass][cls].ensure(sizeof(DminItem) * std::max<size_t>(1, v.size())));
            if (!v.empty())
                BHIP(b, hipMemcpy(b->d_items[pass][cls].p, v.data(), sizeof(DminItem) * v.size(),
                                  hipMemcpyHostToDevice));
        }
    snapshot(b);
    b->planned = true;
    b->stepped = false;
    return MPPI_OK;
}

int persistent_block(int pass) { return pass == 0 ? 256 : 128; }  // lanes per pose tile

// One workgroup per resident slot of the chip (every slot pulls items until
// the queue is empty), never more than there are items.
int persistent_grid(mppi_batch b, int pass, int cls, size_t n_items) {
    return static_cast<int>(std::min<size_t>(n_items, static_cast<size_t>(b->resident[pass][cls])));
}

// The register classes of a pass run one after the other on the batch's
// stream.  (Running them concurrently on forked streams was measured 1%
// slower on the 64-scene batch, 104.1 against 103.1 ms per distance pass on
// one device: the classes' workgroups then share compute units from the
// start instead of only in each class's tail.)
int launch_dmin_pass(mppi_batch b, int pass) {
    for (const int cls : b->cls_order[pass]) {
        const auto& v = b->items[pass][cls];
        BHIP(b, launch_dmin_persistent(cls, persistent_block(pass), persistent_grid(b, pass, cls, v.size()),
                                       b->d_sdm.as<SceneDmin>(), b->d_items[pass][cls].as<DminItem>(),
                                       static_cast<int>(v.size()), b->d_counters.as<int>() + DMIN_CLASSES * pass + cls,
                                       b->stream));
    }
    return MPPI_OK;
}

// The whole batched cycle on b->stream (eager, or recorded into a graph).
int enqueue_step(mppi_batch b) {
    const int n = b->n;
    SceneStep* ds = b->d_steps.as<SceneStep>();
    SceneBufs* db = b->d_bufs.as<SceneBufs>();
    BHIP(b, hipMemcpyAsync(b->d_steps.p, b->h_steps, sizeof(SceneStep) * n, hipMemcpyHostToDevice,
                           b->stream));
    BHIP(b, launch_batch_reset(b->d_counters.as<int>(), 2 * DMIN_CLASSES, b->stream));
    BHIP(b, launch_rollout_batched(ds, db, b->d_blk_roll.as<int2>(),
                                   static_cast<int>(b->blk_roll.size()), b->stream));
    const bool timed = b->prof && !b->capturing;
    if (timed) BHIP(b, hipEventRecord(b->ev0, b->stream));
    if (int rc = launch_dmin_pass(b, 0)) return rc;
    if (timed) BHIP(b, hipEventRecord(b->ev1, b->stream));
    b->prof_pending = timed;
    BHIP(b, launch_cost_batched(ds, db, b->d_blk_roll.as<int2>(),
                                static_cast<int>(b->blk_roll.size()), b->stream));
    BHIP(b, launch_update_batched(ds, db, b->d_blk_upd.as<int2>(),
                                  static_cast<int>(b->blk_upd.size()), b->stream));
    BHIP(b, launch_nominal_batched(ds, db, n, b->stream));
    if (int rc = launch_dmin_pass(b, 1)) return rc;
    BHIP(b, launch_finalize_batched(ds, db, n, b->stream));
    BHIP(b, hipMemcpyAsync(b->h_out, b->d_out.p, sizeof(float) * OUT_FLOATS * n, hipMemcpyDeviceToHost,
                           b->stream));
    return MPPI_OK;
}

int fill_steps(mppi_batch b, const float* q0, float* dU, const uint64_t* seeds,
               const uint64_t* steps) {
    for (int s = 0; s < b->n; ++s) {
        SceneStep& S = b->h_steps[s];
        S.P = b->args[s];
        for (int k = 0; k < 3; ++k) S.P.q0[k] = q0[3 * s + k];
        S.P.seed = seeds[s];
        S.P.step = steps[s];
        S.P.stream = b->noise_stream[s];
        S.P.n_path = b->scenes[s]->n_path;  // guidance may change between steps
        S.U = dU + b->u_off[s];
    }
    return MPPI_OK;
}

// Enqueue one batched step (eagerly, or as a replay of the captured graph)
// and the copy of the result records to pinned host memory; no host sync.
int batch_launch(mppi_batch b, const float* q0, float* dU, const uint64_t* seeds,
                 const uint64_t* steps, int use_graph) {
    if (!q0 || !dU || !seeds || !steps) return bfail(b, MPPI_E_ARG, "NULL argument");
    if (!snapshot_matches(b))
        return bfail(b, MPPI_E_STATE, "a scene's points or footprint changed: call mppi_batch_refresh");
    fill_steps(b, q0, dU, seeds, steps);
    if (use_graph) {
        if (!b->exec) {
            BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
            b->capturing = true;
            const int rc = enqueue_step(b);
            b->capturing = false;
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(b->stream, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            BHIP(b, e);
            b->graph = graph;
            BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        }
        BHIP(b, hipGraphLaunch(b->exec, b->stream));
    } else {
        if (int rc = enqueue_step(b)) return rc;
    }
    return MPPI_OK;
}

// Commands and validation flags of the last step (after the stream synced).
void batch_collect(mppi_batch b, float* u_out, int* valid_out) {
    if (b->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b->ev0, b->ev1) == hipSuccess) {
            b->prof_ms += ms;
            b->prof_n += 1;
        }
        b->prof_pending = false;
    }
    if (!u_out) return;
    for (int s = 0; s < b->n; ++s) {
        for (int k = 0; k < b->prms[s].nu; ++k) u_out[3 * s + k] = b->h_out[OUT_FLOATS * s + k];
        for (int k = b->prms[s].nu; k < 3; ++k) u_out[3 * s + k] = 0.0f;
        if (valid_out) valid_out[s] = b->h_out[OUT_FLOATS * s + 3] != 0.0f;
    }
}

}  // namespace

extern "C" {

int mppi_batch_create(mppi_batch* out, const mppi_ctx* scenes, const mppi_params* prms, int n,
                      void* hip_stream) {
    if (!out) return bfail(nullptr, MPPI_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 4096 || !scenes || !prms) return bfail(nullptr, MPPI_E_ARG, "need 1..4096 scenes");
    const int dev = scenes[0] ? scenes[0]->device : -1;
    for (int s = 0; s < n; ++s) {
        if (!scenes[s]) return bfail(nullptr, MPPI_E_ARG, "scene %d is NULL", s);
        if (scenes[s]->device != dev) return bfail(nullptr, MPPI_E_ARG, "scenes on different devices");
        if (int rc = check_params(scenes[s], &prms[s]))
            return bfail(nullptr, rc, "scene %d: %s", s, scenes[s]->err.c_str());
    }
    mppi_batch b = new mppi_batch_s;
    b->device = dev;
    b->n = n;
    b->scenes.assign(scenes, scenes + n);
    b->prms.assign(prms, prms + n);
    b->u_off.assign(n + 1, 0);
    b->noise_stream.assign(n, 0);
    const float zero3[3] = {0.f, 0.f, 0.f};
    for (int s = 0; s < n; ++s) {
        b->args.push_back(make_args(scenes[s], &prms[s], zero3, 0, 0));
        b->u_off[s + 1] = b->u_off[s] + prms[s].T * prms[s].nu;
    }
    DeviceGuard g(dev);
    hipError_t e = hipSuccess;
    if (hip_stream) {
        b->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        b->own_stream = e == hipSuccess;
    }
    if (e == hipSuccess) e = b->d_steps.ensure(sizeof(SceneStep) * n);
    if (e == hipSuccess) e = b->d_counters.ensure(sizeof(int) * 2 * DMIN_CLASSES);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_steps), sizeof(SceneStep) * n, 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_out), sizeof(float) * OUT_FLOATS * n, 0);
    if (e != hipSuccess) {
        mppi_batch_destroy(b);
        return bfail(nullptr, MPPI_E_HIP, "batch setup: %s", hipGetErrorString(e));
    }
    // default plan: about 2^22 point-primitive pairs per queue item
    if (int rc = plan(b, 0.0)) {
        std::string m = b->err;
        mppi_batch_destroy(b);
        return bfail(nullptr, rc, "%s", m.c_str());
    }
    *out = b;
    return MPPI_OK;
}

int mppi_batch_destroy(mppi_batch b) {
    if (!b) return MPPI_OK;
    {
        DeviceGuard g(b->device);
        if (b->stream) (void)hipStreamSynchronize(b->stream);
        drop_graph(b);
        DevBuf* bufs[] = {&b->arena, &b->d_steps, &b->d_bufs, &b->d_sdm, &b->d_blk_roll,
                          &b->d_blk_upd, &b->d_counters, &b->d_out};
        for (DevBuf* x : bufs) x->release();
        for (auto& pass : b->d_items)
            for (DevBuf& x : pass) x.release();
        if (b->h_steps) (void)hipHostFree(b->h_steps);
        if (b->h_out) (void)hipHostFree(b->h_out);
        if (b->ev0) (void)hipEventDestroy(b->ev0);
        if (b->ev1) (void)hipEventDestroy(b->ev1);
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
    }
    delete b;
    return MPPI_OK;
}

const char* mppi_batch_last_error(mppi_batch b) { return b ? b->err.c_str() : g_create_error.c_str(); }

int mppi_batch_u_offsets(mppi_batch b, int* offsets) {
    if (!b || !offsets) return MPPI_E_ARG;
    for (int s = 0; s <= b->n; ++s) offsets[s] = b->u_off[s];
    return MPPI_OK;
}

int mppi_batch_refresh(mppi_batch b) {
    if (!b) return MPPI_E_ARG;
    DeviceGuard g(b->device);
    return plan(b, b->work_target);
}

int mppi_batch_set_work(mppi_batch b, double work_per_item) {
    if (!b) return MPPI_E_ARG;
    if (!(work_per_item >= 0.0) || work_per_item > 1e15)
        return bfail(b, MPPI_E_ARG, "work_per_item must be >= 0 and finite");
    DeviceGuard g(b->device);
    return plan(b, work_per_item);
}

int mppi_step_batched(mppi_batch b, const float* q0, float* dU, const uint64_t* seeds,
                      const uint64_t* steps, float* u_out, int* valid_out, int use_graph) {
    if (!b) return MPPI_E_ARG;
    if (!u_out) return bfail(b, MPPI_E_ARG, "NULL argument");
    DeviceGuard g(b->device);
    if (int rc = batch_launch(b, q0, dU, seeds, steps, use_graph)) return rc;
    BHIP(b, hipStreamSynchronize(b->stream));
    batch_collect(b, u_out, valid_out);
    b->stepped = true;
    return MPPI_OK;
}

int mppi_batch_set_profiling(mppi_batch b, int enable) {
    if (!b) return MPPI_E_ARG;
    DeviceGuard g(b->device);
    if (enable && !b->ev0) {
        BHIP(b, hipEventCreate(&b->ev0));
        BHIP(b, hipEventCreate(&b->ev1));
    }
    b->prof = enable != 0;
    b->prof_pending = false;
    b->prof_ms = 0.0;
    b->prof_n = 0;
    return MPPI_OK;
}

int mppi_batch_get_profile(mppi_batch b, double* ms, long long* launches) {
    if (!b || !ms || !launches) return MPPI_E_ARG;
    *ms = b->prof_ms;
    *launches = b->prof_n;
    return MPPI_OK;
}

int mppi_batch_nominal_costs(mppi_batch b, float* J_out) {
    if (!b || !J_out) return MPPI_E_ARG;
    for (int s = 0; s < b->n; ++s) J_out[s] = b->h_out[OUT_FLOATS * s + 4];
    return MPPI_OK;
}

int mppi_batch_scene_diag(mppi_batch b, int scene, const mppi_diag* diag) {
    if (!b) return MPPI_E_ARG;
    if (!diag || scene < 0 || scene >= b->n) return bfail(b, MPPI_E_ARG, "need a diag and 0 <= scene < %d", b->n);
    if (diag->argmin || diag->w || diag->u)
        return bfail(b, MPPI_E_ARG, "the batch keeps no argmin, weights or sampled controls");
    if (!b->stepped) return bfail(b, MPPI_E_STATE, "no batched step since the last plan");
    DeviceGuard g(b->device);
    const mppi_params& P = b->prms[scene];
    const SceneDiag d{diag->d_min, diag->poses, diag->eps, diag->J, diag->U_upd, diag->d_nom, diag->J_nom};
    BHIP(b, launch_scene_diag(b->bufs[scene], P.K, b->args[scene].Kpad, P.T, P.nu, d, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return MPPI_OK;
}

int mppi_batch_autotune(mppi_batch b, int reps, double* out_work_per_item) {
    if (!b) return MPPI_E_ARG;
    if (reps < 1) reps = 3;
    DeviceGuard g(b->device);
    // poses of one cycle around zero nominals
    std::vector<float> zeros(3 * b->n, 0.f);
    std::vector<uint64_t> seeds(b->n, 0x7E57ull), stepv(b->n, 0);
    DevBuf dU;
    BHIP(b, dU.ensure(sizeof(float) * std::max(1, b->u_off[b->n])));
    BHIP(b, hipMemsetAsync(dU.p, 0, sizeof(float) * std::max(1, b->u_off[b->n]), b->stream));
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    // candidates: 2^16 .. 2^26 pairs per item
    std::vector<double> cand;
    for (int lg = 16; lg <= 26; ++lg) cand.push_back(std::ldexp(1.0, lg));
    std::vector<float> best(cand.size(), 1e30f);
    int rc = MPPI_OK;
    // time `launches` passes of plan w (rollout poses regenerated per plan);
    // returns the mean of all but the first launch
    auto time_plan = [&](double w, int launches, float* mean_ms) -> int {
        if (int r = plan(b, w)) return r;
        fill_steps(b, zeros.data(), dU.as<float>(), seeds.data(), stepv.data());
        hipError_t e = hipMemcpyAsync(b->d_steps.p, b->h_steps, sizeof(SceneStep) * b->n,
                                      hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = launch_rollout_batched(b->d_steps.as<SceneStep>(), b->d_bufs.as<SceneBufs>(),
                                       b->d_blk_roll.as<int2>(), static_cast<int>(b->blk_roll.size()),
                                       b->stream);
        if (e != hipSuccess) return bfail(b, MPPI_E_HIP, "autotune: %s", hipGetErrorString(e));
        float total = 0.f;
        for (int k = 0; k < launches; ++k) {
            e = launch_batch_reset(b->d_counters.as<int>(), 2 * DMIN_CLASSES, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            if (e != hipSuccess) return bfail(b, MPPI_E_HIP, "autotune timing: %s", hipGetErrorString(e));
            if (int r = launch_dmin_pass(b, 0)) return r;
            e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) return bfail(b, MPPI_E_HIP, "autotune timing: %s", hipGetErrorString(e));
            if (k > 0) total += ms;  // the first launch is a warm-up
        }
        *mean_ms = launches > 1 ? total / (launches - 1) : 0.f;
        return MPPI_OK;
    };
    // warm the clocks up on the default plan, then time every candidate in a
    // forward and a backward sweep and keep each one's faster sweep, so
    // clock ramps do not favour the later candidates
    float warm = 0.f;
    rc = time_plan(0.0, 8, &warm);
    for (int sweep = 0; sweep < 2 && rc == MPPI_OK; ++sweep)
        for (size_t n = 0; n < cand.size() && rc == MPPI_OK; ++n) {
            const size_t ci = sweep == 0 ? n : cand.size() - 1 - n;
            float ms = 0.f;
            rc = time_plan(cand[ci], reps + 1, &ms);
            if (rc == MPPI_OK) best[ci] = std::min(best[ci], ms);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dU.release();
    if (rc) return rc;
    size_t bi = 0;
    for (size_t ci = 1; ci < cand.size(); ++ci)
        if (best[ci] < best[bi]) bi = ci;
    if (int r2 = plan(b, cand[bi])) return r2;
    if (out_work_per_item) *out_work_per_item = cand[bi];
    return MPPI_OK;
}

int mppi_batch_info(mppi_batch b, long long* items_main, long long* items_validation,
                    double* work_per_item) {
    if (!b) return MPPI_E_ARG;
    long long m = 0, v = 0;
    for (int cls = 0; cls < DMIN_CLASSES; ++cls) {
        m += static_cast<long long>(b->items[0][cls].size());
        v += static_cast<long long>(b->items[1][cls].size());
    }
    if (items_main) *items_main = m;
    if (items_validation) *items_validation = v;
    if (work_per_item) *work_per_item = b->work_per_item;
    return MPPI_OK;
}

// ------------------------------------------------------------ hybrid modes

int mppi_hybrid_create(mppi_hybrid* out, mppi_ctx scene, const mppi_params* modes, int n_modes,
                       void* hip_stream) {
    if (!out) return bfail(nullptr, MPPI_E_ARG, "out is NULL");
    *out = nullptr;
    if (!scene || !modes || n_modes < 1 || n_modes > HYB_MAX_MODES)
        return bfail(nullptr, MPPI_E_ARG, "need a context and 1..%d modes", HYB_MAX_MODES);
    for (int m = 0; m < n_modes; ++m)
        if (!modes[m].validate)
            return bfail(nullptr, MPPI_E_ARG, "mode %d: hybrid selection needs validation on", m);
    std::vector<mppi_ctx> sc(n_modes, scene);
    mppi_batch b = nullptr;
    if (int rc = mppi_batch_create(&b, sc.data(), modes, n_modes, hip_stream)) return rc;
    // every mode draws its own noise: Philox stream word = mode index
    for (int m = 0; m < n_modes; ++m) b->noise_stream[m] = static_cast<uint64_t>(m);
    mppi_hybrid h = new mppi_hybrid_s;
    h->b = b;
    h->n = n_modes;
    for (int m = 0; m < n_modes; ++m) {
        h->model[m] = modes[m].model;
        h->nu[m] = modes[m].nu;
    }
    DeviceGuard g(b->device);
    hipError_t e = h->d_res.ensure(sizeof(float) * OUT_FLOATS);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&h->h_res), sizeof(float) * OUT_FLOATS, 0);
    if (e != hipSuccess) {
        mppi_hybrid_destroy(h);
        return bfail(nullptr, MPPI_E_HIP, "hybrid setup: %s", hipGetErrorString(e));
    }
    *out = h;
    return MPPI_OK;
}

int mppi_hybrid_destroy(mppi_hybrid h) {
    if (!h) return MPPI_OK;
    if (h->b) {
        DeviceGuard g(h->b->device);
        if (h->b->stream) (void)hipStreamSynchronize(h->b->stream);
        h->d_res.release();
        if (h->h_res) (void)hipHostFree(h->h_res);
        mppi_batch_destroy(h->b);
    }
    delete h;
    return MPPI_OK;
}

const char* mppi_hybrid_last_error(mppi_hybrid h) {
    return h ? (h->err.empty() && h->b ? h->b->err.c_str() : h->err.c_str()) : g_create_error.c_str();
}

mppi_batch mppi_hybrid_batch(mppi_hybrid h) { return h ? h->b : nullptr; }

int mppi_hybrid_step(mppi_hybrid h, const float q0[3], float* dU, uint64_t seed, uint64_t step,
                     const mppi_hybrid_params* hp, int* m_prev, int* tau_cool, float u_out[3],
                     int* stopped, float* J_modes, int* valid_modes, int use_graph) {
    if (!h) return MPPI_E_ARG;
    h->err.clear();
    auto hfail = [&](int code, const char* msg) {
        h->err = msg;
        return code;
    };
    if (!q0 || !dU || !hp || !m_prev || !tau_cool || !u_out) return hfail(MPPI_E_ARG, "NULL argument");
    if (*m_prev < 0 || *m_prev >= h->n) return hfail(MPPI_E_ARG, "m_prev out of range");
    if (*tau_cool < 0 || hp->cool_max < 0) return hfail(MPPI_E_ARG, "negative cooldown");
    if (!(hp->lambda_switch >= 0.0f) || !(hp->v_min >= 0.0f) || !(hp->w_min >= 0.0f))
        return hfail(MPPI_E_ARG, "lambda_switch, v_min and w_min must be >= 0");
    mppi_batch b = h->b;
    DeviceGuard g(b->device);
    std::vector<float> q(3 * h->n);
    std::vector<uint64_t> seeds(h->n, seed), steps(h->n, step);
    for (int m = 0; m < h->n; ++m)
        for (int k = 0; k < 3; ++k) q[3 * m + k] = q0[k];
    if (int rc = batch_launch(b, q.data(), dU, seeds.data(), steps.data(), use_graph)) return rc;
    HybridArgs a{};
    a.n_modes = h->n;
    a.m_prev = *m_prev;
    a.tau_cool = *tau_cool;
    a.cool_max = hp->cool_max;
    a.lambda_switch = hp->lambda_switch;
    a.v_min = hp->v_min;
    a.w_min = hp->w_min;
    a.noise_v = hp->noise_v;
    a.noise_w = hp->noise_w;
    for (int m = 0; m < h->n; ++m) {
        a.model[m] = h->model[m];
        a.nu[m] = h->nu[m];
    }
    BHIP(b, launch_hybrid_select(b->d_out.as<float>(), a, h->d_res.as<float>(), b->stream));
    BHIP(b, hipMemcpyAsync(h->h_res, h->d_res.p, sizeof(float) * OUT_FLOATS, hipMemcpyDeviceToHost,
                           b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    batch_collect(b, nullptr, nullptr);
    b->stepped = true;
    for (int k = 0; k < 3; ++k) u_out[k] = h->h_res[k];
    *m_prev = static_cast<int>(h->h_res[3]);
    *tau_cool = static_cast<int>(h->h_res[4]);
    for (int m = 0; m < h->n; ++m) {
        if (J_modes) J_modes[m] = b->h_out[OUT_FLOATS * m + 4];
        if (valid_modes) valid_modes[m] = b->h_out[OUT_FLOATS * m + 3] != 0.0f;
    }
    if (stopped) *stopped = h->h_res[5] != 0.0f;
    return MPPI_OK;
}

}  // extern "C"
