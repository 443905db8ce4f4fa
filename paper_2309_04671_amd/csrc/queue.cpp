// Continuous-batching shot queue: admission by resident-byte budget, a
// first-fit arena sub-allocator, batched chunks of leapfrog steps replayed
// from captured HIP graphs, and a worker thread that admits and retires
// shots between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "log.h"

namespace {

using sp::fail;
using sp::ok;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// Planes per block of a shot that shares its launch with other shots.  A
// lone grid is split along z as far as it needs to fill the GPU (a small
// grid into chunks shorter than this); in a batch the other shots supply
// that parallelism, and short, equal chunks keep the launch's tail short.
// Measured on a saturating batch of the four served shapes: 16 beats the
// lone-grid split by 1.8 % in capacity, 8 and 12 lose to the re-read
// start-up planes, 24 and longer to the tail.  A shot alone in its launch
// keeps its own split.  The z-split never changes a point's arithmetic.
constexpr int QUEUE_ZCHUNK = 16;

// Same block -> tile map as the single-grid kernels (contiguous per XCD).
int xcd_tile_host(int bid, int n) {
    const int xcd = bid & 7, loc = bid >> 3, q = n >> 3, r = n & 7;
    return xcd * q + std::min(xcd, r) + loc;
}

// First-fit allocator over byte offsets; adjacent free ranges coalesce.
class Arena {
  public:
    void reset(int64_t base, int64_t size) {
        free_.clear();
        if (size > 0) free_[base] = size;
    }
    int64_t alloc(int64_t n) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const int64_t off = it->first, rem = it->second - n;
                free_.erase(it);
                if (rem > 0) free_[off + n] = rem;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t largest() const {
        int64_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    std::map<int64_t, int64_t> free_;
};

struct Shot {
    uint64_t id = 0;
    sp_shot_desc d;
    sp_grid g, gv;
    sp::TileCfg tile;
    sp::SweepArgs base;          // validated arguments without per-step fields (own z-split)
    int nblk = 0;                // blocks at the batch z-split (at least those of base)
    sp::SweepArgs run;           // base with the z-split of the current composition
    int nblk_run = 0;
    int64_t bytes = 0, off = -1;
    int64_t step = 0;
    int state = SP_SHOT_QUEUED, error = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    char *f0 = nullptr, *f1 = nullptr;   // the two wavefield allocations
    float *v = nullptr, *meta = nullptr;
    uint32_t *nonfinite = nullptr;       // device flag: a non-finite value was computed
    void *cur = nullptr, *prev = nullptr;
    hipEvent_t ready = nullptr;          // caller's inputs produced
    bool fresh = false;                  // admitted, not yet initialised on the device
    bool blown = false;                  // the last chunk computed a non-finite value
};

struct Group {
    int dtype;
    sp::TileCfg tile;
    std::vector<Shot *> members;     // stable pointers into the queue's shot map
    int nblk = 0, nrec = 0;
    int64_t off_table = 0, off_rmap = 0, off_args = 0, off_recs = 0;
};

}  // namespace

struct sp_queue {
    sp_queue_cfg cfg;
    bool fake = false, eager = false;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;    // graph capture only (never executes work)
    hipEvent_t chunk_done = nullptr;
    char *ctrl_dev = nullptr;            // control part of the arena (tables, per-step args)
    int64_t ctrl_bytes = 0, budget = 0, resident = 0;
    char *pinned = nullptr;              // host staging of the control part
    Arena arena;
    uint64_t fail_ticket = 0;            // test hook: fail this ticket at admission
    uint64_t nonfinite_ticket = 0;       // test hook (fake executor): this ticket blows up
    uint32_t *flags_host = nullptr;      // pinned: the active shots' non-finite flags

    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<uint64_t> pending;
    std::map<uint64_t, Shot> shots;
    std::vector<uint64_t> active;
    uint64_t next_id = 1;
    bool stopping = false;
    std::thread worker;

    // current composition
    std::vector<uint64_t> comp_ids;
    int comp_k = 0;
    std::vector<Group> groups;
    int64_t dyn_off = 0, dyn_bytes = 0;  // per-chunk region of the control part
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Two wavefields, v, then the slab records (FP16/BF16) followed by the
// shot's non-finite flag.
int64_t shot_bytes(const sp_grid &g, const sp_grid &gv) {
    return 2 * align256(g.bytes) + align256(gv.bytes) + align256(sp_wave_meta_bytes(&g) + 16);
}

// Control bytes needed by a composition (upper bound used at admission).
int64_t ctrl_need(const std::vector<const Shot *> &set, int k) {
    int64_t blocks = 0, recs = 0;
    for (auto *s : set) {
        blocks += s->nblk;
        recs += s->d.nrec;
    }
    const int64_t n = (int64_t)set.size();
    return align256(blocks * 8) * 3 + align256(recs * 8) * 3 +
           (int64_t)k * n * (align256(sizeof(sp::SweepArgs)) + align256(sizeof(sp::RecArgs))) + 4096;
}

void release_shot(sp_queue *q, Shot &s) {
    if (s.off >= 0) {
        q->arena.release(s.off, s.bytes);
        q->resident -= s.bytes;
        s.off = -1;
    }
}

void destroy_graph(sp_queue *q) {
    if (q->exec) (void)hipGraphExecDestroy(q->exec);
    if (q->graph) (void)hipGraphDestroy(q->graph);
    q->exec = nullptr;
    q->graph = nullptr;
}

// Lay out the control part for the active set and k steps per chunk and
// upload the static tables (the chunk graph is captured by the first chunk).
int rebuild(sp_queue *q, const std::vector<Shot *> &act, int k) {
    destroy_graph(q);
    q->groups.clear();
    for (Shot *sp_ : act) {
        Shot &s = *sp_;
        Group *gp = nullptr;
        for (auto &g : q->groups)
            if (g.dtype == s.g.dtype && g.tile.tx == s.tile.tx && g.tile.ty == s.tile.ty &&
                g.tile.ry == s.tile.ry)
                gp = &g;
        if (!gp) {
            q->groups.push_back(Group());
            gp = &q->groups.back();
            gp->dtype = s.g.dtype;
            gp->tile = s.tile;
        }
        gp->members.push_back(&s);
        gp->nrec += std::max(0, s.d.nrec);
    }
    for (auto &g : q->groups) {
        for (Shot *m : g.members) {
            const int zc = g.members.size() > 1 ? std::min(QUEUE_ZCHUNK, m->g.nz) : m->base.zchunk;
            m->run = m->base;
            m->run.zchunk = zc;
            m->run.nzc = (m->g.nz + zc - 1) / zc;
            m->nblk_run = m->run.tiles_x * m->run.tiles_y * m->run.nzc;
            g.nblk += m->nblk_run;
        }
    }
    // static part: tables and receiver maps; dynamic part: per-step arguments
    int64_t off = 0;
    for (auto &g : q->groups) {
        g.off_table = off;
        off += align256((int64_t)g.nblk * 8);
        g.off_rmap = off;
        off += align256((int64_t)g.nrec * 8);
    }
    const int64_t static_end = off;
    q->dyn_off = off;
    for (auto &g : q->groups) {
        g.off_args = off;
        off += align256((int64_t)k * g.members.size() * sizeof(sp::SweepArgs));
        g.off_recs = off;
        off += align256((int64_t)k * g.members.size() * sizeof(sp::RecArgs));
    }
    q->dyn_bytes = off - q->dyn_off;
    if (off > q->ctrl_bytes) return fail(SP_ENOMEM, "queue: control data exceeds its arena part");
    if (sp::log_on()) {
        int blocks = 0;
        for (auto &g : q->groups) blocks += g.nblk;
        sp::log_line("queue: composition of %zu shots in %zu groups, %d blocks per step, %d steps per chunk",
                     act.size(), q->groups.size(), blocks, k);
    }
    q->comp_ids.clear();
    for (Shot *a : act) q->comp_ids.push_back(a->id);
    q->comp_k = k;
    if (q->fake) return SP_OK;

    for (auto &g : q->groups) {
        int2 *table = reinterpret_cast<int2 *>(q->pinned + g.off_table);
        std::vector<int> prefix(1, 0);
        for (Shot *m : g.members) prefix.push_back(prefix.back() + m->nblk_run);
        for (int b = 0; b < g.nblk; ++b) {
            const int gl = xcd_tile_host(b, g.nblk);
            const int m = int(std::upper_bound(prefix.begin(), prefix.end(), gl) - prefix.begin()) - 1;
            table[b] = make_int2(m, gl - prefix[m]);
        }
        int2 *rmap = reinterpret_cast<int2 *>(q->pinned + g.off_rmap);
        int r = 0;
        for (size_t m = 0; m < g.members.size(); ++m)
            for (int i = 0; i < g.members[m]->d.nrec; ++i) rmap[r++] = make_int2((int)m, i);
    }
    if (static_end > 0) {
        hipError_t e = hipMemcpyAsync(q->ctrl_dev, q->pinned, static_end, hipMemcpyHostToDevice, q->stream);
        if (e != hipSuccess) return fail(SP_EDEVICE, "queue: table upload: %s", hipGetErrorString(e));
    }
    return SP_OK;
}

// The k steps of the current composition: per step and group one batched
// sweep and one batched receiver launch, reading their arguments from the
// control part.
hipError_t launch_steps(sp_queue *q, int k, hipStream_t st) {
    hipError_t e = hipSuccess;
    for (int i = 0; i < k && e == hipSuccess; ++i) {
        for (auto &g : q->groups) {
            const int nm = (int)g.members.size();
            auto *args = reinterpret_cast<const sp::SweepArgs *>(q->ctrl_dev + g.off_args) + (int64_t)i * nm;
            auto *table = reinterpret_cast<const int2 *>(q->ctrl_dev + g.off_table);
            e = sp::launch_sweep_batch(sp::MODE_WAVE, g.dtype, g.tile, args, table, g.nblk, st);
            if (e == hipSuccess && g.nrec > 0) {
                auto *recs = reinterpret_cast<const sp::RecArgs *>(q->ctrl_dev + g.off_recs) + (int64_t)i * nm;
                auto *rmap = reinterpret_cast<const int2 *>(q->ctrl_dev + g.off_rmap);
                e = sp::launch_record_batch(g.dtype, recs, rmap, g.nrec, st);
            }
            if (e != hipSuccess) break;
        }
    }
    return e;
}

// Capture the current composition's chunk into a graph on the capture-only
// stream (nothing executes there).  Called right after the composition's
// first chunk was launched directly, so the capture and instantiation run
// on the host while the GPU works, off the chunks' critical path.  On
// failure the composition keeps launching directly.
void capture_chunk(sp_queue *q, int k) {
    hipError_t e = hipStreamBeginCapture(q->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return;
    e = launch_steps(q, k, q->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(q->cap_stream, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&q->exec, graph, nullptr, nullptr, 0);
    q->graph = graph;
    if (e != hipSuccess) destroy_graph(q);
}

// Fill the per-step arguments of the next k steps and run them.
int run_chunk(sp_queue *q, int k) {
    if (q->fake) {
        for (auto &g : q->groups)
            for (Shot *m : g.members) m->blown = m->id == q->nonfinite_ticket;
        return SP_OK;
    }
    for (auto &g : q->groups) {
        const int nm = (int)g.members.size();
        auto *args = reinterpret_cast<sp::SweepArgs *>(q->pinned + g.off_args);
        auto *recs = reinterpret_cast<sp::RecArgs *>(q->pinned + g.off_recs);
        for (int m = 0; m < nm; ++m) {
            Shot &s = *g.members[m];
            void *cur = s.cur, *prev = s.prev;
            for (int i = 0; i < k; ++i) {
                const int64_t n = s.step + i;
                sp::SweepArgs &a = args[(int64_t)i * nm + m];
                a = s.run;
                a.v = s.v + s.gv.origin;
                sp::step_args(a, &s.g, cur, prev, prev, s.meta, n, s.d.src_amp, s.d.nsrc);
                a.nonfinite = s.nonfinite;
                sp::RecArgs &r = recs[(int64_t)i * nm + m];
                r.field = a.out;
                r.scale = s.meta ? a.meta.s_out : nullptr;
                r.xyz = s.d.rec_xyz;
                r.traces = s.d.nrec > 0 ? s.d.traces + n * s.d.nrec : nullptr;
                r.sy = s.g.pitch_x;
                r.sz = s.g.pitch_x * s.g.pitch_y;
                r.nx = s.g.nx;
                r.ny = s.g.ny;
                r.nz = s.g.nz;
                r.n = s.d.nrec;
                std::swap(cur, prev);
            }
        }
    }
    hipError_t e = hipSuccess;
    if (q->dyn_bytes > 0)
        e = hipMemcpyAsync(q->ctrl_dev + q->dyn_off, q->pinned + q->dyn_off, q->dyn_bytes,
                           hipMemcpyHostToDevice, q->stream);
    // A composition's first chunk is launched directly and its graph
    // captured while that chunk runs; later chunks of the same composition
    // replay the graph.  Short-lived compositions never pay for a capture
    // on the critical path.
    bool capture = false;
    if (e == hipSuccess) {
        if (q->exec) {
            e = hipGraphLaunch(q->exec, q->stream);
        } else {
            e = launch_steps(q, k, q->stream);
            capture = !q->eager;
        }
    }
    if (e == hipSuccess && capture) capture_chunk(q, k);
    // the resident shots' non-finite flags, read back with the chunk
    int nflag = 0;
    for (auto &g : q->groups)
        for (Shot *m : g.members) {
            if (e == hipSuccess)
                e = hipMemcpyAsync(q->flags_host + nflag, m->nonfinite, sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, q->stream);
            ++nflag;
        }
    if (e == hipSuccess) e = hipEventRecord(q->chunk_done, q->stream);
    if (e == hipSuccess) e = hipEventSynchronize(q->chunk_done);
    if (e != hipSuccess) return fail(SP_EDEVICE, "queue: chunk failed: %s", hipGetErrorString(e));
    nflag = 0;
    for (auto &g : q->groups)
        for (Shot *m : g.members) m->blown = q->flags_host[nflag++] != 0;
    return SP_OK;
}

// Zero the admitted shot's fields and records and copy its velocity in.
int init_shot(sp_queue *q, Shot &s) {
    if (q->fake) return SP_OK;
    hipError_t e = hipStreamWaitEvent(q->stream, s.ready, 0);
    if (e == hipSuccess) e = hipMemsetAsync(s.f0, 0, s.g.bytes, q->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s.f1, 0, s.g.bytes, q->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s.v, 0, s.gv.bytes, q->stream);
    if (e == hipSuccess && s.meta) e = hipMemsetAsync(s.meta, 0, sp_wave_meta_bytes(&s.g), q->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s.nonfinite, 0, sizeof(uint32_t), q->stream);
    if (e == hipSuccess)
        e = sp::launch_pack(s.d.v, s.v + s.gv.origin, s.gv.pitch_x, s.gv.pitch_x * s.gv.pitch_y,
                            s.gv.nx, s.gv.ny, s.gv.nz, q->stream);
    if (e != hipSuccess) return fail(SP_EDEVICE, "queue: shot setup: %s", hipGetErrorString(e));
    return SP_OK;
}

int finish_shot(sp_queue *q, Shot &s) {
    if (q->fake || !s.d.final_out) return SP_OK;
    float *scale = nullptr;
    if (s.meta) {
        const int nslab = (s.g.nz + SP_SLAB - 1) / SP_SLAB;
        scale = s.meta + ((s.step % 4 + 4) % 4) * 2 * nslab;
    }
    hipError_t e = sp::launch_unpack(s.g.dtype, static_cast<char *>(s.cur) + s.g.origin * s.g.elem_bytes,
                                     scale, s.d.final_out, s.g.pitch_x, s.g.pitch_x * s.g.pitch_y,
                                     s.g.nx, s.g.ny, s.g.nz, q->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(q->stream);
    if (e != hipSuccess) return fail(SP_EDEVICE, "queue: final field: %s", hipGetErrorString(e));
    return SP_OK;
}

void worker_main(sp_queue *q) {
    if (!q->fake) (void)hipSetDevice(q->device);
    for (;;) {
        std::vector<Shot *> fresh, act;
        std::vector<uint64_t> act_ids;
        int k = 0;
        {
            std::unique_lock<std::mutex> lk(q->mu);
            // admission (FIFO): stop at the first shot that does not fit yet
            while (!q->stopping && !q->pending.empty() && (int)q->active.size() < q->cfg.max_slots) {
                Shot &s = q->shots[q->pending.front()];
                if (q->resident + s.bytes > q->budget) break;
                std::vector<const Shot *> cand;
                for (uint64_t id : q->active) cand.push_back(&q->shots[id]);
                cand.push_back(&s);
                if (ctrl_need(cand, q->cfg.chunk_steps) > q->ctrl_bytes) break;
                const int64_t off = q->arena.alloc(s.bytes);
                if (off < 0) break;
                q->pending.pop_front();
                s.off = off;
                q->resident += s.bytes;
                s.t_admit = now_s();
                if (s.id == q->fail_ticket) {
                    s.state = SP_SHOT_FAILED;
                    s.error = SP_EDEVICE;
                    s.t_done = now_s();
                    release_shot(q, s);
                    q->cv_done.notify_all();
                    continue;
                }
                char *base = static_cast<char *>(q->cfg.arena) + off;
                s.f0 = base;
                s.f1 = base + align256(s.g.bytes);
                s.v = reinterpret_cast<float *>(base + 2 * align256(s.g.bytes));
                char *rec = base + 2 * align256(s.g.bytes) + align256(s.gv.bytes);
                s.meta = s.g.dtype == SP_F32 ? nullptr : reinterpret_cast<float *>(rec);
                s.nonfinite = reinterpret_cast<uint32_t *>(rec + sp_wave_meta_bytes(&s.g));
                s.cur = s.f1;
                s.prev = s.f0;
                s.state = SP_SHOT_RUNNING;
                sp::log_line("queue: admit ticket %llu, %dx%dx%d dtype %d, %d steps, %lld bytes "
                             "(resident %lld of %lld), waited %.4f s",
                             (unsigned long long)s.id, s.g.nx, s.g.ny, s.g.nz, s.g.dtype, s.d.nsteps,
                             (long long)s.bytes, (long long)q->resident, (long long)q->budget,
                             s.t_admit - s.t_submit);
                q->active.push_back(s.id);
                fresh.push_back(&s);
            }
            if (q->active.empty()) {
                if (q->stopping) break;
                q->cv.wait(lk);
                continue;
            }
            k = q->cfg.chunk_steps;
            for (uint64_t id : q->active) {
                Shot &s = q->shots.at(id);
                act.push_back(&s);
                act_ids.push_back(id);
                k = (int)std::min<int64_t>(k, s.d.nsteps - s.step);
            }
        }
        // device work outside the lock (submissions and polls proceed
        // meanwhile); only the worker touches these shots' device state and
        // map nodes are stable, so the pointers stay valid
        int err = SP_OK;
        for (Shot *s : fresh)
            if (!err) err = init_shot(q, *s);
        if (!err && (q->comp_ids != act_ids || q->comp_k != k)) err = rebuild(q, act, k);
        if (!err) err = run_chunk(q, k);
        {
            std::lock_guard<std::mutex> lk(q->mu);
            std::vector<uint64_t> still;
            for (uint64_t id : q->active) {
                Shot &s = q->shots[id];
                if (err) {
                    s.state = SP_SHOT_FAILED;
                    s.error = err;
                } else {
                    s.step += k;
                    if (k % 2) std::swap(s.cur, s.prev);
                    if (s.blown) {
                        // blown up: its neighbours in the batch are unaffected
                        // (no shot reads another's memory)
                        s.state = SP_SHOT_FAILED;
                        s.error = SP_ENUMERIC;
                    } else if (s.step >= s.d.nsteps) {
                        const int e = finish_shot(q, s);
                        s.state = e ? SP_SHOT_FAILED : SP_SHOT_DONE;
                        s.error = e;
                    }
                }
                if (s.state == SP_SHOT_RUNNING) {
                    still.push_back(id);
                } else {
                    s.t_done = now_s();
                    release_shot(q, s);
                    sp::log_line("queue: ticket %llu %s (error %d) after %lld steps, latency %.4f s",
                                 (unsigned long long)s.id, s.state == SP_SHOT_DONE ? "done" : "failed",
                                 s.error, (long long)s.step, s.t_done - s.t_submit);
                }
            }
            q->active.swap(still);
            q->cv_done.notify_all();
        }
    }
}

}  // namespace

extern "C" {

int64_t sp_shot_bytes(const sp_shot_desc *d) {
    if (!d) return -1;
    sp_grid g, gv;
    if (sp_grid_init(d->nx, d->ny, d->nz, SP_HALO, d->dtype, &g) != SP_OK) return -1;
    if (sp_grid_init(d->nx, d->ny, d->nz, SP_HALO, SP_F32, &gv) != SP_OK) return -1;
    return shot_bytes(g, gv);
}

int sp_queue_create(const sp_queue_cfg *cfg, sp_queue **out) {
    if (!cfg || !out) return fail(SP_EINVAL, "sp_queue_create: NULL argument");
    if (!cfg->arena || cfg->arena_bytes <= 0) return fail(SP_EINVAL, "sp_queue_create: no arena");
    if (reinterpret_cast<uintptr_t>(cfg->arena) & 255u) return fail(SP_EINVAL, "sp_queue_create: arena must be 256-byte aligned");
    if (cfg->max_slots < 1 || cfg->chunk_steps < 1 || cfg->chunk_steps > 1024)
        return fail(SP_EINVAL, "sp_queue_create: max_slots >= 1 and 1 <= chunk_steps <= 1024");
    if (cfg->flags & ~(SP_QUEUE_EAGER | SP_QUEUE_FAKE)) return fail(SP_EINVAL, "sp_queue_create: unknown flags");
    sp_queue *q = new sp_queue();
    q->cfg = *cfg;
    q->fake = (cfg->flags & SP_QUEUE_FAKE) != 0;
    q->eager = (cfg->flags & SP_QUEUE_EAGER) != 0;
    // control part: per-step arguments and tables, at the start of the arena
    q->ctrl_bytes = align256(std::min<int64_t>(std::max<int64_t>(cfg->arena_bytes / 16, 16 << 20), 256 << 20));
    if (q->ctrl_bytes >= cfg->arena_bytes) {
        delete q;
        return fail(SP_EINVAL, "sp_queue_create: arena smaller than its control part");
    }
    const int64_t shot_space = cfg->arena_bytes - q->ctrl_bytes;
    q->budget = cfg->budget_bytes > 0 ? std::min(cfg->budget_bytes, shot_space) : shot_space;
    q->arena.reset(q->ctrl_bytes, shot_space);
    q->ctrl_dev = static_cast<char *>(cfg->arena);
    if (const char *e = std::getenv("SP_TEST_FAIL_TICKET")) q->fail_ticket = std::strtoull(e, nullptr, 10);
    if (const char *e = std::getenv("SP_TEST_NONFINITE_TICKET"))
        q->nonfinite_ticket = std::strtoull(e, nullptr, 10);
    if (!q->fake) {
        hipError_t e = hipGetDevice(&q->device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&q->chunk_done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&q->pinned), q->ctrl_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&q->flags_host),
                              sizeof(uint32_t) * (size_t)cfg->max_slots, hipHostMallocDefault);
        if (e != hipSuccess) {
            if (q->pinned) (void)hipHostFree(q->pinned);
            if (q->cap_stream) (void)hipStreamDestroy(q->cap_stream);
            if (q->stream) (void)hipStreamDestroy(q->stream);
            if (q->chunk_done) (void)hipEventDestroy(q->chunk_done);
            delete q;
            return fail(SP_EDEVICE, "sp_queue_create: %s", hipGetErrorString(e));
        }
    }
    q->worker = std::thread(worker_main, q);
    *out = q;
    return ok();
}

int sp_submit(sp_queue *q, const sp_shot_desc *d, uint64_t *ticket) {
    if (!q || !d || !ticket) return fail(SP_EINVAL, "sp_submit: NULL argument");
    Shot s;
    s.d = *d;
    if (sp_grid_init(d->nx, d->ny, d->nz, SP_HALO, d->dtype, &s.g) != SP_OK ||
        sp_grid_init(d->nx, d->ny, d->nz, SP_HALO, SP_F32, &s.gv) != SP_OK)
        return fail(SP_EINVAL, "sp_submit: bad shot shape or dtype");
    if (d->nsteps < 1) return fail(SP_EINVAL, "sp_submit: nsteps must be >= 1");
    if (!q->fake && !d->v) return fail(SP_EINVAL, "sp_submit: v is NULL");
    if (d->nrec < 0 || (d->nrec > 0 && (!d->rec_xyz || !d->traces)))
        return fail(SP_EINVAL, "sp_submit: receiver arrays");
    sp_sources src;
    src.n = d->nsrc;
    std::memcpy(src.xyz, d->src_xyz, sizeof src.xyz);
    src.amp = d->src_amp;
    src.amp_stride = d->nsrc;
    sp_receivers rec{d->nrec, d->rec_xyz, d->traces, d->nrec};
    // validate with a stand-in velocity pointer; the real one lives in the arena
    if (int e = sp::prep_wave("sp_submit", &s.g, &d->coeffs, d->dt, d->dx, &s.gv,
                              reinterpret_cast<const float *>(q->cfg.arena), d->nsrc ? &src : nullptr,
                              d->nrec ? &rec : nullptr, &s.base, &s.tile))
        return e;
    {
        // blocks at the larger of the two z-splits (alone: its own; batched: QUEUE_ZCHUNK)
        const int zb = std::min(QUEUE_ZCHUNK, s.g.nz), zs = s.base.zchunk;
        s.nblk = s.base.tiles_x * s.base.tiles_y *
                 std::max((s.g.nz + zb - 1) / zb, (s.g.nz + zs - 1) / zs);
    }
    if (!sp::batch_supported(s.tile))
        return fail(SP_EUNSUPPORTED, "sp_submit: tile configuration %dx%dx%d is not batched",
                    s.tile.tx, s.tile.ty, s.tile.ry);
    s.bytes = shot_bytes(s.g, s.gv);
    {
        std::vector<const Shot *> one{&s};
        if (s.bytes > q->budget || ctrl_need(one, q->cfg.chunk_steps) > q->ctrl_bytes)
            return fail(SP_EBUDGET, "sp_submit: shot needs %lld bytes, budget %lld",
                        (long long)s.bytes, (long long)q->budget);
    }
    if (!q->fake) {
        hipError_t e = hipEventCreateWithFlags(&s.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(s.ready, static_cast<hipStream_t>(q->cfg.stream));
        if (e != hipSuccess) return fail(SP_EDEVICE, "sp_submit: %s", hipGetErrorString(e));
    }
    s.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(q->mu);
        if (q->stopping) return fail(SP_EINVAL, "sp_submit: queue is shutting down");
        s.id = q->next_id++;
        *ticket = s.id;
        q->pending.push_back(s.id);
        q->shots.emplace(s.id, s);
    }
    q->cv.notify_all();
    return ok();
}

int sp_poll(sp_queue *q, uint64_t ticket, sp_shot_status *st) {
    if (!q || !st) return fail(SP_EINVAL, "sp_poll: NULL argument");
    std::lock_guard<std::mutex> lk(q->mu);
    auto it = q->shots.find(ticket);
    if (it == q->shots.end()) return fail(SP_EINVAL, "sp_poll: unknown ticket %llu", (unsigned long long)ticket);
    const Shot &s = it->second;
    st->state = s.state;
    st->error = s.error;
    st->steps_done = s.step;
    st->t_submit = s.t_submit;
    st->t_admit = s.t_admit;
    st->t_done = s.t_done;
    if (s.state == SP_SHOT_DONE || s.state == SP_SHOT_FAILED) return ok();
    return SP_EPENDING;
}

int sp_queue_drain(sp_queue *q) {
    if (!q) return fail(SP_EINVAL, "sp_queue_drain: NULL queue");
    std::unique_lock<std::mutex> lk(q->mu);
    q->cv_done.wait(lk, [q] {
        for (auto &kv : q->shots)
            if (kv.second.state == SP_SHOT_QUEUED || kv.second.state == SP_SHOT_RUNNING) return false;
        return true;
    });
    return ok();
}

int sp_queue_destroy(sp_queue *q) {
    if (!q) return fail(SP_EINVAL, "sp_queue_destroy: NULL queue");
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->stopping = true;
        for (uint64_t id : q->pending) {
            Shot &s = q->shots[id];
            s.state = SP_SHOT_FAILED;
            s.error = SP_EINVAL;
            s.t_done = now_s();
        }
        q->pending.clear();
    }
    q->cv.notify_all();
    q->worker.join();
    if (!q->fake) {
        destroy_graph(q);
        for (auto &kv : q->shots)
            if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
        (void)hipStreamSynchronize(q->stream);
        (void)hipEventDestroy(q->chunk_done);
        (void)hipStreamDestroy(q->cap_stream);
        (void)hipStreamDestroy(q->stream);
        (void)hipHostFree(q->pinned);
        (void)hipHostFree(q->flags_host);
    }
    delete q;
    return ok();
}

}  // extern "C"
