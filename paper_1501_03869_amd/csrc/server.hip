// Frame server: resident delay tables and continuous batching of frames of
// different geometries (the paper's offline table build once per geometry,
// online back projection per frame, Section III).
//
// Threads:
//  * scheduler - forms a batch from the queued frames whose map is ready, up
//    to max_batch frames and as device memory allows, uploads them, launches
//    one mixed-geometry gather (descriptor per frame) and the image downloads,
//    and records an event.  Up to max_inflight batches are on the device at
//    once, alternating between two streams so uploads overlap gathers.
//  * completion - waits for batch events in order, time-stamps the frames
//    (latency = submit -> image in pinned host memory) and frees their slots.
//  * builder - runs table builds (pat_eikonal_tables, then the 16.16
//    conversion when configured) on a stream and context of its own, so new
//    speed maps are prepared while frames keep flowing.
// Admission: a frame needs a free slot (max_slots frames submitted and not
// yet collected by pat_server_wait) and, to be launched, device memory; a
// map needs room for its table and build working set inside the HBM budget,
// after evicting idle ready maps (least recently used first).  An evicted map
// is rebuilt when a frame for it arrives.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pat_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

enum MapState { MAP_BUILDING = 0, MAP_READY = 1, MAP_FAILED = 2, MAP_EVICTED = 3, MAP_QUEUED = 4 };
enum FrameState { FR_QUEUED = 0, FR_INFLIGHT = 1, FR_DONE = 2, FR_FAILED = 3 };

struct Map {
    int id = 0;
    int state = MAP_QUEUED;
    int nx = 0, ny = 0, nz = 0;  // nz = 0: a 2-D map
    double h = 0;
    std::vector<float> speed;
    std::vector<double> sxy;     // [S][2], or [S][3] for a 3-D map
    std::vector<int32_t> pix;
    int S = 0, P = 0, N = 0;
    double t0 = 0, dt = 0;
    void *d_table = nullptr;
    size_t table_bytes = 0;
    size_t build_bytes = 0;  // reserved while a build runs
    int refs = 0;            // queued + in-flight frames
    uint64_t last_use = 0;
    int err = PAT_OK;
    bool removed = false;
};

struct Frame {
    uint64_t ticket = 0;
    int map_id = 0;
    int sig_fmt = PAT_SIG_F32;
    float scale = 1.0f;
    void *h_in = nullptr;
    size_t in_bytes = 0;
    float *h_out = nullptr;
    size_t out_bytes = 0;
    void *d_in = nullptr;
    float *d_out = nullptr;
    double t_submit = 0, t_done = 0;
    int state = FR_QUEUED;
    int rc = PAT_OK;
    int64_t gathers = 0;
};

struct BatchSlot {
    int idx = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    pat_bp_desc *h_desc = nullptr;   // pinned
    pat_bp_desc *d_desc = nullptr;
    int desc_cap = 0;
    std::vector<Frame *> frames;
    bool busy = false;
};

// Exact-size free lists of device or pinned host buffers.
struct Pool {
    bool host = false;
    std::multimap<size_t, void *> free_;
    size_t free_bytes = 0;
    void *get(size_t bytes) {
        auto it = free_.find(bytes);
        if (it == free_.end()) return nullptr;
        void *p = it->second;
        free_.erase(it);
        free_bytes -= bytes;
        return p;
    }
    void put(void *p, size_t bytes) {
        if (!p) return;
        free_.emplace(bytes, p);
        free_bytes += bytes;
    }
    void release_all() {
        for (auto &kv : free_) {
            if (host) (void)hipHostFree(kv.second);
            else (void)hipFree(kv.second);
        }
        free_.clear();
        free_bytes = 0;
    }
};

}  // namespace

struct pat_server {
    pat_ctx *user_ctx = nullptr;
    int device = 0;
    pat_server_config cfg{};
    pat_ctx *build_ctx = nullptr;
    hipStream_t build_stream = nullptr;
    hipStream_t streams[2] = { nullptr, nullptr };  // batch streams, alternating

    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_build, cv_slot;
    bool stop = false;
    bool hold = false;  // queued frames wait until released

    std::unordered_map<int, std::unique_ptr<Map>> maps;
    int next_map = 1;
    std::deque<int> build_queue;
    std::unordered_map<uint64_t, std::unique_ptr<Frame>> frames;
    std::deque<Frame *> pending;
    uint64_t next_ticket = 1;
    uint64_t lru_clock = 0;
    int frames_in_system = 0;

    std::vector<BatchSlot> slots;
    std::deque<BatchSlot *> inflight;

    Pool dev_pool, host_pool;
    size_t fault_bytes = 0;    // injected allocation failure threshold (PAT_FAULT_ALLOC_BYTES; 0 = off)
    size_t used = 0;           // device bytes in use or pooled (tables, frames, scratch, build reservation)
    size_t build_scratch = 0;  // bytes held by the builder's context

    // statistics
    int64_t st_submitted = 0, st_done = 0, st_refused = 0, st_batches = 0, st_batch_frames = 0, st_builds = 0,
            st_evictions = 0, st_gathers = 0;
    double win_start = 0, win_last = 0;
    int64_t win_frames = 0, win_gathers = 0;
    std::vector<float> lat_us;  // ring of recent latencies
    size_t lat_next = 0;

    std::thread th_sched, th_done, th_build;
    std::atomic<int> thread_error{ PAT_OK };

    // ---- memory (caller holds mu)
    bool evict_one() {
        Map *victim = nullptr;
        for (auto &kv : maps) {
            Map *m = kv.second.get();
            if (m->state == MAP_READY && m->refs == 0 && (!victim || m->last_use < victim->last_use)) victim = m;
        }
        if (!victim) return false;
        dev_pool.put(victim->d_table, victim->table_bytes);
        victim->d_table = nullptr;
        victim->state = MAP_EVICTED;
        ++st_evictions;
        return true;
    }
    // make room for `bytes` more inside the budget: drop pooled buffers, then idle maps
    bool make_room(size_t bytes) {
        if (used + bytes <= cfg.hbm_budget_bytes) return true;
        if (dev_pool.free_bytes) {
            used -= dev_pool.free_bytes;
            dev_pool.release_all();
            if (used + bytes <= cfg.hbm_budget_bytes) return true;
        }
        while (used + bytes > cfg.hbm_budget_bytes) {
            if (!evict_one()) return false;
            used -= dev_pool.free_bytes;
            dev_pool.release_all();
        }
        return true;
    }
    void *dev_alloc(size_t bytes) {
        void *p = dev_pool.get(bytes);
        if (p) return p;  // pooled bytes are already counted in `used`
        if (!make_room(bytes)) return nullptr;
        if (fault_bytes && bytes >= fault_bytes) return nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        used += bytes;
        return p;
    }
    void dev_free(void *p, size_t bytes) { dev_pool.put(p, bytes); }
    void *host_alloc(size_t bytes) {
        void *p = host_pool.get(bytes);
        if (p) return p;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }

    // working memory pat_eikonal_tables will allocate in the builder's context
    // beyond what it already holds (its buffers only grow)
    size_t map_build_bytes(const Map &m) const {
        const size_t n = (size_t)m.nx * m.ny * std::max(m.nz, 1);
        const size_t tiles = m.nz > 0 ? (size_t)((m.nx + 7) / 8) * ((m.ny + 7) / 8) * ((m.nz + 7) / 8)
                                      : (size_t)((m.nx + 31) / 32) * ((m.ny + 31) / 32);
        const size_t maps_per_chunk = std::min<size_t>(m.S, std::max<size_t>(1, (8ull << 30) / (n * 4)));
        const size_t est = maps_per_chunk * n * 4 + n * 4 + 4 * tiles * maps_per_chunk * 4 + maps_per_chunk * 512 + 4096;
        return est > build_scratch ? est - build_scratch : 0;
    }
    // bytes a build also allocates through the pool: speed map, pixels, table(s)
    size_t map_pool_bytes(const Map &m) const {
        size_t b = (size_t)m.nx * m.ny * std::max(m.nz, 1) * 4 + (size_t)m.P * 4 + table_bytes(m);
        if (cfg.table_fmt != PAT_TABLE_F32) b += (size_t)m.S * m.P * 4;  // the float32 table it is made from
        return b;
    }
    // bytes of a map's resident table in the configured format
    size_t table_bytes(const Map &m) const {
        return cfg.table_fmt == PAT_TABLE_R16 ? pat_r16_bytes(m.S, m.P) : (size_t)m.S * m.P * 4;
    }
    // queue a (re)build of an evicted map if its memory can be found
    void ensure_building(Map *m) {
        if (m->state != MAP_EVICTED) return;
        const size_t resv = map_build_bytes(*m);
        if (!make_room(resv + map_pool_bytes(*m))) return;
        m->build_bytes = resv;
        used += resv;
        m->state = MAP_QUEUED;
        build_queue.push_back(m->id);
        cv_build.notify_all();
    }

    void record_latency(double us) {
        if (lat_us.size() < 65536) lat_us.push_back((float)us);
        else lat_us[lat_next++ % lat_us.size()] = (float)us;
    }

    void fail_frame(Frame *f, int rc) {
        f->state = FR_FAILED;
        f->rc = rc;
        auto it = maps.find(f->map_id);
        if (it != maps.end()) it->second->refs--;
    }

    void scheduler();
    void completion();
    void builder();
};

// ----------------------------------------------------------------------------- builder

void pat_server::builder() {
    (void)hipSetDevice(device);
    for (;;) {
        Map *m = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_build.wait(lk, [&] { return stop || !build_queue.empty(); });
            if (stop) return;
            const int id = build_queue.front();
            build_queue.pop_front();
            auto it = maps.find(id);
            if (it == maps.end() || it->second->removed) continue;
            m = it->second.get();
            m->state = MAP_BUILDING;
        }
        int rc = PAT_OK;
        const size_t n = (size_t)m->nx * m->ny * std::max(m->nz, 1);
        void *d_speed = nullptr, *d_pix = nullptr, *d_f32 = nullptr, *d_out = nullptr;
        const size_t t32 = (size_t)m->S * m->P * 4;  // float32 table
        const size_t tb = table_bytes(*m);           // resident table
        const bool convert = cfg.table_fmt != PAT_TABLE_F32;
        {
            std::lock_guard<std::mutex> lk(mu);
            d_speed = dev_alloc(n * 4);
            d_pix = dev_alloc((size_t)m->P * 4);
            d_out = dev_alloc(tb);
            if (convert) d_f32 = dev_alloc(t32);
            if (!d_speed || !d_pix || !d_out || (convert && !d_f32)) rc = PAT_ENOMEM;
        }
        if (rc == PAT_OK) {
            float *table32 = static_cast<float *>(convert ? d_f32 : d_out);
            if (hipMemcpyAsync(d_speed, m->speed.data(), n * 4, hipMemcpyHostToDevice, build_stream) != hipSuccess ||
                hipMemcpyAsync(d_pix, m->pix.data(), (size_t)m->P * 4, hipMemcpyHostToDevice, build_stream) != hipSuccess)
                rc = PAT_EDEVICE;
            if (rc == PAT_OK)
                rc = m->nz > 0 ? pat_eikonal_tables_3d(build_ctx, static_cast<float *>(d_speed), m->nx, m->ny, m->nz, m->h,
                                                       m->sxy.data(), m->S, static_cast<int32_t *>(d_pix), m->P,
                                                       table32, build_stream)
                               : pat_eikonal_tables(build_ctx, static_cast<float *>(d_speed), m->nx, m->ny, m->h,
                                                    m->sxy.data(), m->S, static_cast<int32_t *>(d_pix), m->P, table32,
                                                    build_stream);
            if (rc == PAT_OK && cfg.table_fmt == PAT_TABLE_Q16)
                rc = pat_table_to_q16(build_ctx, table32, (int64_t)m->S * m->P, m->t0, m->dt, m->N,
                                      static_cast<uint32_t *>(d_out), build_stream);
            if (rc == PAT_OK && cfg.table_fmt == PAT_TABLE_R16)
                rc = pat_table_to_r16(build_ctx, table32, m->S, m->P, m->t0, m->dt, m->N, d_out, build_stream);
            if (rc == PAT_OK && hipStreamSynchronize(build_stream) != hipSuccess) rc = PAT_EDEVICE;
        }
        size_t scratch = build_ctx->eik_tq.bytes + build_ctx->eik_f.bytes + build_ctx->eik_flags.bytes +
                         build_ctx->eik_lists.bytes + build_ctx->eik_seeds.bytes + build_ctx->eik_count.bytes;
        {
            std::lock_guard<std::mutex> lk(mu);
            dev_free(d_speed, n * 4);
            dev_free(d_pix, (size_t)m->P * 4);
            if (d_f32) dev_free(d_f32, t32);
            // the builder's context keeps its working maps for the next build
            if (scratch > build_scratch) {
                used += scratch - build_scratch;
                build_scratch = scratch;
            }
            used -= std::min(used, m->build_bytes);
            m->build_bytes = 0;
            if (rc == PAT_OK && !m->removed) {
                m->d_table = d_out;
                m->table_bytes = tb;
                m->state = MAP_READY;
                m->last_use = ++lru_clock;
                ++st_builds;
            } else {
                if (d_out) dev_free(d_out, tb);
                m->state = MAP_FAILED;
                m->err = rc ? rc : PAT_ENOTFOUND;
                // frames waiting for this map cannot be served
                for (auto it = pending.begin(); it != pending.end();) {
                    if ((*it)->map_id == m->id) {
                        fail_frame(*it, m->err);
                        it = pending.erase(it);
                    } else {
                        ++it;
                    }
                }
                cv_done.notify_all();
                cv_slot.notify_all();
            }
        }
        cv_sched.notify_all();
    }
}

// ----------------------------------------------------------------------------- scheduler

void pat_server::scheduler() {
    (void)hipSetDevice(device);
    for (;;) {
        BatchSlot *slot = nullptr;
        std::vector<Frame *> batch;
        int batch_fmt = -1;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) return;
                slot = nullptr;
                for (auto &s : slots)
                    if (!s.busy) { slot = &s; break; }
                bool ready = false;
                for (Frame *f : pending) {
                    auto it = maps.find(f->map_id);
                    if (it == maps.end()) continue;
                    if (it->second->state == MAP_READY) ready = true;
                    else if (it->second->state == MAP_EVICTED) ensure_building(it->second.get());
                }
                if (slot && ready && !hold) break;
                cv_sched.wait_for(lk, std::chrono::milliseconds(50));
            }
            // take ready frames in arrival order while device memory allows; one
            // launch gathers one signal format, that of the oldest ready frame
            batch_fmt = -1;
            for (auto it = pending.begin(); it != pending.end() && (int)batch.size() < cfg.max_batch;) {
                Frame *f = *it;
                Map *m = maps[f->map_id].get();
                if (m->state != MAP_READY || (batch_fmt >= 0 && f->sig_fmt != batch_fmt)) { ++it; continue; }
                batch_fmt = f->sig_fmt;
                f->d_in = dev_alloc(f->in_bytes);
                f->d_out = f->d_in ? static_cast<float *>(dev_alloc(f->out_bytes)) : nullptr;
                if (!f->d_in || !f->d_out) {
                    if (f->d_in) dev_free(f->d_in, f->in_bytes);
                    f->d_in = nullptr;
                    f->d_out = nullptr;
                    break;
                }
                m->last_use = ++lru_clock;
                f->state = FR_INFLIGHT;
                batch.push_back(f);
                it = pending.erase(it);
            }
            if (batch.empty()) {  // memory is full: wait for a completion
                cv_sched.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            slot->busy = true;
        }
        // descriptors
        int rc = PAT_OK;
        const int nd = (int)batch.size();
        int blocks = 0;
        std::vector<pat_bp_desc> desc((size_t)nd);
        {
            std::lock_guard<std::mutex> lk(mu);
            for (int i = 0; i < nd; ++i) {
                Frame *f = batch[(size_t)i];
                Map *m = maps[f->map_id].get();
                pat_bp_desc &d = desc[(size_t)i];
                const int nb = pat_px_frame_shape(&d, m->S, m->P, m->N, m->t0, m->dt);
                d.tab = static_cast<const uint32_t *>(m->d_table);
                d.sig = f->d_in;
                d.w = nullptr;
                d.img = f->d_out;
                d.scale = f->sig_fmt == PAT_SIG_F16 ? f->scale : 1.0f;
                d.block_begin = blocks;
                blocks += nb;
            }
        }
        if (nd > slot->desc_cap) {
            if (slot->h_desc) (void)hipHostFree(slot->h_desc);
            if (slot->d_desc) (void)hipFree(slot->d_desc);
            slot->h_desc = nullptr;
            slot->d_desc = nullptr;
            slot->desc_cap = 0;
            if (hipHostMalloc((void **)&slot->h_desc, sizeof(pat_bp_desc) * nd, hipHostMallocDefault) != hipSuccess ||
                hipMalloc((void **)&slot->d_desc, sizeof(pat_bp_desc) * nd) != hipSuccess)
                rc = PAT_ENOMEM;
            else
                slot->desc_cap = nd;
        }
        if (rc == PAT_OK) {
            std::memcpy(slot->h_desc, desc.data(), sizeof(pat_bp_desc) * nd);
            hipStream_t st = slot->stream;
            for (Frame *f : batch)
                if (hipMemcpyAsync(f->d_in, f->h_in, f->in_bytes, hipMemcpyHostToDevice, st) != hipSuccess) rc = PAT_EDEVICE;
            if (hipMemcpyAsync(slot->d_desc, slot->h_desc, sizeof(pat_bp_desc) * nd, hipMemcpyHostToDevice, st) != hipSuccess)
                rc = PAT_EDEVICE;
            if (rc == PAT_OK) rc = pat_launch_px_multi(slot->d_desc, nd, blocks, cfg.table_fmt, batch_fmt, st);
            for (Frame *f : batch)
                if (rc == PAT_OK && hipMemcpyAsync(f->h_out, f->d_out, f->out_bytes, hipMemcpyDeviceToHost, st) != hipSuccess)
                    rc = PAT_EDEVICE;
            if (rc == PAT_OK && hipEventRecord(slot->ev, st) != hipSuccess) rc = PAT_EDEVICE;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            if (rc != PAT_OK) {
                // nothing reached the device in a usable state: fail these frames
                (void)hipStreamSynchronize(slot->stream);
                for (Frame *f : batch) {
                    dev_free(f->d_in, f->in_bytes);
                    dev_free(f->d_out, f->out_bytes);
                    f->d_in = nullptr;
                    f->d_out = nullptr;
                    fail_frame(f, rc);
                }
                slot->busy = false;
                thread_error = rc;
                cv_done.notify_all();
                cv_slot.notify_all();
                continue;
            }
            slot->frames = std::move(batch);
            ++st_batches;
            st_batch_frames += nd;
            inflight.push_back(slot);
        }
        cv_done.notify_all();
    }
}

// ----------------------------------------------------------------------------- completion

void pat_server::completion() {
    (void)hipSetDevice(device);
    for (;;) {
        BatchSlot *slot = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_done.wait(lk, [&] { return stop || !inflight.empty(); });
            if (stop && inflight.empty()) return;
            slot = inflight.front();
        }
        const hipError_t e = hipEventSynchronize(slot->ev);
        const double t = now_s();
        {
            std::lock_guard<std::mutex> lk(mu);
            inflight.pop_front();
            for (Frame *f : slot->frames) {
                dev_free(f->d_in, f->in_bytes);
                dev_free(f->d_out, f->out_bytes);
                f->d_in = nullptr;
                f->d_out = nullptr;
                auto it = maps.find(f->map_id);
                if (it != maps.end()) it->second->refs--;
                if (e != hipSuccess) {
                    f->state = FR_FAILED;
                    f->rc = PAT_EDEVICE;
                    continue;
                }
                f->state = FR_DONE;
                f->t_done = t;
                ++st_done;
                st_gathers += f->gathers;
                if (win_frames == 0 && win_start == 0) win_start = f->t_submit;
                ++win_frames;
                win_gathers += f->gathers;
                win_last = t;
                record_latency((t - f->t_submit) * 1e6);
            }
            slot->frames.clear();
            slot->busy = false;
        }
        cv_done.notify_all();
        cv_slot.notify_all();
        cv_sched.notify_all();
    }
}

// ----------------------------------------------------------------------------- C ABI

extern "C" int pat_server_create_ex(pat_ctx *ctx, const pat_server_config *cfg, pat_server **out) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (!out) return pat_fail(PAT_EINVAL, "out is NULL");
    *out = nullptr;
    pat_server_config c{};
    if (cfg) c = *cfg;
    if (c.table_fmt != PAT_TABLE_F32 && c.table_fmt != PAT_TABLE_Q16 && c.table_fmt != PAT_TABLE_R16)
        return pat_fail(PAT_EINVAL, "bad table format");
    if (c.max_batch <= 0) c.max_batch = 64;
    if (c.max_inflight <= 0) c.max_inflight = 2;
    if (c.max_slots <= 0) c.max_slots = 1024;
    if (c.max_batch > 4096 || c.max_inflight > 8) return pat_fail(PAT_EINVAL, "max_batch <= 4096, max_inflight <= 8");
    if (c.hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        PAT_HIP(hipMemGetInfo(&fr, &tot));
        c.hbm_budget_bytes = (size_t)(0.8 * (double)fr);
    }
    std::unique_ptr<pat_server> s(new (std::nothrow) pat_server());
    if (!s) return pat_fail(PAT_ENOMEM, "host allocation failed");
    s->user_ctx = ctx;
    s->device = ctx->device;
    s->cfg = c;
    s->host_pool.host = true;
    s->fault_bytes = pat_env_fault_alloc_bytes();
    if ((rc = pat_ctx_create(ctx->device, &s->build_ctx))) return rc;
    auto cleanup = [&]() {
        for (auto &sl : s->slots)
            if (sl.ev) (void)hipEventDestroy(sl.ev);
        for (hipStream_t st : s->streams)
            if (st) (void)hipStreamDestroy(st);
        if (s->build_stream) (void)hipStreamDestroy(s->build_stream);
        pat_ctx_destroy(s->build_ctx);
    };
    if (hipStreamCreateWithFlags(&s->build_stream, hipStreamNonBlocking) != hipSuccess) {
        cleanup();
        return pat_fail(PAT_EDEVICE, "stream creation failed");
    }
    s->slots.resize((size_t)c.max_inflight);
    for (int i = 0; i < 2; ++i)
        if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) {
            cleanup();
            return pat_fail(PAT_EDEVICE, "stream creation failed");
        }
    for (int i = 0; i < c.max_inflight; ++i) {
        BatchSlot &sl = s->slots[(size_t)i];
        sl.idx = i;
        sl.stream = s->streams[i % 2];
        if (hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
            cleanup();
            return pat_fail(PAT_EDEVICE, "event creation failed");
        }
    }
    s->th_sched = std::thread([p = s.get()] { p->scheduler(); });
    s->th_done = std::thread([p = s.get()] { p->completion(); });
    s->th_build = std::thread([p = s.get()] { p->builder(); });
    *out = s.release();
    return PAT_OK;
}

extern "C" int pat_server_create(pat_ctx *ctx, size_t hbm_budget_bytes, pat_server **out) {
    pat_server_config c{};
    c.hbm_budget_bytes = hbm_budget_bytes;
    c.table_fmt = PAT_TABLE_F32;
    return pat_server_create_ex(ctx, &c, out);
}

extern "C" int pat_server_destroy(pat_server *s) {
    if (!s) return PAT_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        // let in-flight batches finish
        s->cv_slot.wait(lk, [&] { return s->inflight.empty(); });
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
    s->cv_build.notify_all();
    s->th_sched.join();
    s->th_done.join();
    s->th_build.join();
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    for (auto &sl : s->slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.h_desc) (void)hipHostFree(sl.h_desc);
        if (sl.d_desc) (void)hipFree(sl.d_desc);
    }
    for (auto &kv : s->maps)
        if (kv.second->d_table) (void)hipFree(kv.second->d_table);
    for (auto &kv : s->frames) {
        Frame *f = kv.second.get();
        if (f->h_in) s->host_pool.put(f->h_in, f->in_bytes);
        if (f->h_out) s->host_pool.put(f->h_out, f->out_bytes);
        if (f->d_in) (void)hipFree(f->d_in);
        if (f->d_out) (void)hipFree(f->d_out);
    }
    s->dev_pool.release_all();
    s->host_pool.release_all();
    if (s->build_stream) (void)hipStreamDestroy(s->build_stream);
    pat_ctx_destroy(s->build_ctx);
    delete s;
    return PAT_OK;
}

// A 2-D map (nz = 0, sensors [S][2]) or a 3-D map (nz >= 1, sensors [S][3]).
static int add_map(pat_server *s, const float *h_speed, int nx, int ny, int nz, double h, const double *h_sensor,
                   int S, const int32_t *h_pix, int P, double t0, double dt, int N, int *map_id) {
    if (!s || !map_id) return pat_fail(PAT_EINVAL, "null argument");
    const bool vol = nz > 0;
    const bool grid_ok = vol ? nx >= 1 && ny >= 1 && (long long)nx * ny * nz >= 2 && (long long)nx * ny * nz <= (1LL << 30)
                             : nx >= 2 && ny >= 2;
    if (!grid_ok || !(h > 0) || S <= 0 || P <= 0 || N < 4 || !(dt > 0) || !std::isfinite(t0))
        return pat_fail(PAT_EINVAL, "bad map geometry");
    if (!pat_px_multi_eligible(PAT_SIG_F16, S, P, N))
        return pat_fail(PAT_EINVAL, "map too large for the frame server (S*P or S*N beyond 32-bit offsets)");
    if (!h_speed || !h_sensor || !h_pix) return pat_fail(PAT_EINVAL, "null map data");
    if (s->cfg.table_fmt != PAT_TABLE_F32 && N > 65535)
        return pat_fail(PAT_EINVAL, "16.16 and 16-bit tables need N <= 65535");
    const size_t n = (size_t)nx * ny * (vol ? nz : 1);
    for (size_t k = 0; k < n; ++k)
        if (!(std::isfinite(h_speed[k]) && h_speed[k] > 0)) return pat_fail(PAT_EINVAL, "speed must be finite and > 0");
    for (int p = 0; p < P; ++p)
        if (h_pix[p] < 0 || (size_t)h_pix[p] >= n) return pat_fail(PAT_EINVAL, "pixel index out of range");
    const int dim = vol ? 3 : 2;
    const int ext[3] = { nx, ny, vol ? nz : 1 };
    for (int i = 0; i < S; ++i)
        for (int a = 0; a < dim; ++a) {
            const double g = (h_sensor[dim * i + a] + 0.5 * (ext[a] - 1) * h) / h;
            if (!(g >= 0 && g <= ext[a] - 1)) return pat_fail(PAT_EINVAL, "sensor outside the grid");
        }
    auto m = std::make_unique<Map>();
    m->nx = nx; m->ny = ny; m->nz = vol ? nz : 0; m->h = h; m->S = S; m->P = P; m->N = N; m->t0 = t0; m->dt = dt;
    m->speed.assign(h_speed, h_speed + n);
    m->sxy.assign(h_sensor, h_sensor + (size_t)dim * S);
    m->pix.assign(h_pix, h_pix + P);
    std::lock_guard<std::mutex> lk(s->mu);
    const size_t resv = s->map_build_bytes(*m);
    const size_t need = resv + s->map_pool_bytes(*m);
    if (!s->make_room(need))
        return pat_fail(PAT_EBUSY, "map needs %zu bytes; budget %zu, in use %zu", need, s->cfg.hbm_budget_bytes, s->used);
    m->build_bytes = resv;
    s->used += resv;
    m->id = s->next_map++;
    m->state = MAP_QUEUED;
    *map_id = m->id;
    s->build_queue.push_back(m->id);
    s->maps[m->id] = std::move(m);
    s->cv_build.notify_all();
    return PAT_OK;
}

extern "C" int pat_server_add_map(pat_server *s, const float *h_speed, int nx, int ny, double h,
                                  const double *h_sensor_xy, int S, const int32_t *h_pix, int P, double t0, double dt,
                                  int N, int *map_id) {
    return add_map(s, h_speed, nx, ny, 0, h, h_sensor_xy, S, h_pix, P, t0, dt, N, map_id);
}

extern "C" int pat_server_add_map_3d(pat_server *s, const float *h_speed, int nx, int ny, int nz, double h,
                                     const double *h_sensor_xyz, int S, const int32_t *h_vox, int P, double t0,
                                     double dt, int N, int *map_id) {
    if (nz < 1) return pat_fail(PAT_EINVAL, "bad map geometry");
    return add_map(s, h_speed, nx, ny, nz, h, h_sensor_xyz, S, h_vox, P, t0, dt, N, map_id);
}

extern "C" int pat_server_map_state(pat_server *s, int map_id, int *state) {
    if (!s || !state) return pat_fail(PAT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->maps.find(map_id);
    if (it == s->maps.end() || it->second->removed) return pat_fail(PAT_ENOTFOUND, "unknown map %d", map_id);
    const int st = it->second->state;
    *state = st == MAP_QUEUED ? PAT_MAP_BUILDING : st == MAP_BUILDING ? PAT_MAP_BUILDING
           : st == MAP_READY ? PAT_MAP_READY : st == MAP_EVICTED ? PAT_MAP_EVICTED : PAT_MAP_FAILED;
    return PAT_OK;
}

extern "C" int pat_server_submit(pat_server *s, int map_id, const void *h_frame, int sig_fmt, float scale,
                                 int nonblocking, uint64_t *ticket) {
    if (!s || !h_frame || !ticket) return pat_fail(PAT_EINVAL, "null argument");
    if (sig_fmt != PAT_SIG_F32 && sig_fmt != PAT_SIG_F16) return pat_fail(PAT_EINVAL, "unknown signal format %d", sig_fmt);
    if (sig_fmt == PAT_SIG_F16 && !(std::isfinite(scale) && scale > 0))
        return pat_fail(PAT_EINVAL, "scale must be finite and > 0");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->maps.find(map_id);
    if (it == s->maps.end() || it->second->removed) return pat_fail(PAT_ENOTFOUND, "unknown map %d", map_id);
    Map *m = it->second.get();
    if (m->state == MAP_FAILED) return pat_fail(m->err ? m->err : PAT_EDEVICE, "map %d failed to build", map_id);
    if (!pat_px_multi_eligible(sig_fmt, m->S, m->P, m->N))
        return pat_fail(PAT_EINVAL, "float32 frames of map %d exceed the gather's 32-bit offsets", map_id);
    const size_t esz = sig_fmt == PAT_SIG_F16 ? 2 : 4;
    const size_t in_b = (size_t)m->S * m->N * esz, out_b = (size_t)m->P * 4;
    if (in_b + out_b > s->cfg.hbm_budget_bytes) return pat_fail(PAT_EINVAL, "frame larger than the HBM budget");
    if (s->frames_in_system >= s->cfg.max_slots) {
        if (nonblocking) {
            ++s->st_refused;
            return pat_fail(PAT_EBUSY, "all %d frame slots are in use", s->cfg.max_slots);
        }
        s->cv_slot.wait(lk, [&] { return s->stop || s->frames_in_system < s->cfg.max_slots; });
        if (s->stop) return pat_fail(PAT_EBUSY, "server stopping");
        it = s->maps.find(map_id);
        if (it == s->maps.end() || it->second->removed) return pat_fail(PAT_ENOTFOUND, "unknown map %d", map_id);
        m = it->second.get();
    }
    void *hin = s->host_alloc(in_b);
    void *hout = hin ? s->host_alloc(out_b) : nullptr;
    if (!hin || !hout) {
        if (hin) s->host_pool.put(hin, in_b);
        return pat_fail(PAT_ENOMEM, "pinned host allocation failed");
    }
    std::memcpy(hin, h_frame, in_b);
    auto f = std::make_unique<Frame>();
    f->ticket = s->next_ticket++;
    f->map_id = map_id;
    f->sig_fmt = sig_fmt;
    f->scale = sig_fmt == PAT_SIG_F16 ? scale : 1.0f;
    f->h_in = hin;
    f->in_bytes = in_b;
    f->h_out = static_cast<float *>(hout);
    f->out_bytes = out_b;
    f->t_submit = now_s();
    f->gathers = (int64_t)m->S * m->P;
    *ticket = f->ticket;
    m->refs++;
    s->frames_in_system++;
    s->st_submitted++;
    s->ensure_building(m);  // rebuild an evicted map on demand
    s->pending.push_back(f.get());
    s->frames[f->ticket] = std::move(f);
    lk.unlock();
    s->cv_sched.notify_all();
    return PAT_OK;
}

extern "C" int pat_server_wait(pat_server *s, uint64_t ticket, float *h_img, int timeout_ms) {
    if (!s) return pat_fail(PAT_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->frames.find(ticket);
    if (it == s->frames.end()) return pat_fail(PAT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Frame *f = it->second.get();
    auto finished = [&] { return f->state == FR_DONE || f->state == FR_FAILED; };
    if (timeout_ms < 0) s->cv_done.wait(lk, finished);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished))
        return pat_fail(PAT_ETIMEOUT, "frame %llu not finished after %d ms", (unsigned long long)ticket, timeout_ms);
    int rc = f->rc;
    if (f->state == FR_DONE && h_img) std::memcpy(h_img, f->h_out, f->out_bytes);
    s->host_pool.put(f->h_in, f->in_bytes);
    s->host_pool.put(f->h_out, f->out_bytes);
    s->frames.erase(it);
    s->frames_in_system--;  // the slot is free once the image is collected
    lk.unlock();
    s->cv_slot.notify_all();
    if (rc) return pat_fail(rc, "frame %llu failed", (unsigned long long)ticket);
    return PAT_OK;
}

extern "C" int pat_server_remove_map(pat_server *s, int map_id) {
    if (!s) return pat_fail(PAT_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->maps.find(map_id);
    if (it == s->maps.end() || it->second->removed) return pat_fail(PAT_ENOTFOUND, "unknown map %d", map_id);
    Map *m = it->second.get();
    if (m->refs > 0 || m->state == MAP_BUILDING || m->state == MAP_QUEUED)
        return pat_fail(PAT_EBUSY, "map %d has frames or a build in progress", map_id);
    if (m->d_table) s->dev_free(m->d_table, m->table_bytes);
    m->d_table = nullptr;
    s->maps.erase(it);
    return PAT_OK;
}

extern "C" int pat_server_stats(pat_server *s, pat_stats *out) {
    if (!s || !out) return pat_fail(PAT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    pat_stats r{};
    r.frames_submitted = s->st_submitted;
    r.frames_done = s->st_done;
    r.frames_refused = s->st_refused;
    r.batches = s->st_batches;
    r.builds = s->st_builds;
    r.evictions = s->st_evictions;
    r.mean_batch_frames = s->st_batches ? (double)s->st_batch_frames / s->st_batches : 0.0;
    const double span = s->win_last - s->win_start;
    r.frames_per_s = span > 0 ? s->win_frames / span : 0.0;
    r.gathers_per_s = span > 0 ? s->win_gathers / span : 0.0;
    if (!s->lat_us.empty()) {
        std::vector<float> v = s->lat_us;
        auto pct = [&](double q) {
            const size_t k = std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5));
            std::nth_element(v.begin(), v.begin() + k, v.end());
            return (double)v[k];
        };
        r.latency_p50_us = pct(0.50);
        r.latency_p99_us = pct(0.99);
        r.latency_max_us = *std::max_element(v.begin(), v.end());
    }
    r.bytes_budget = s->cfg.hbm_budget_bytes;
    r.bytes_used = s->used;
    for (auto &kv : s->maps) {
        if (kv.second->state == MAP_READY) {
            r.bytes_tables += kv.second->table_bytes;
            r.maps_ready++;
        } else if (kv.second->state == MAP_BUILDING || kv.second->state == MAP_QUEUED) {
            r.maps_building++;
        }
    }
    r.queue_depth = (int)s->pending.size();
    r.inflight_batches = (int)s->inflight.size();
    *out = r;
    return PAT_OK;
}

extern "C" int pat_server_reset_stats(pat_server *s) {
    if (!s) return pat_fail(PAT_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    s->win_start = 0;
    s->win_last = 0;
    s->win_frames = 0;
    s->win_gathers = 0;
    s->lat_us.clear();
    s->lat_next = 0;
    return PAT_OK;
}

extern "C" int pat_server_hold(pat_server *s, int hold) {
    if (!s) return pat_fail(PAT_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->hold = hold != 0;
    }
    s->cv_sched.notify_all();
    return PAT_OK;
}
