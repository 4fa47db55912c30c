// server.cpp -- streaming block server of liblbf.
//
// Jobs (beam-forming blocks) are queued on the host and admitted in arrival
// order when (a) fewer than max_inflight jobs are on the device and (b) their
// device footprint -- the weights of a not-yet-cached observation, the station
// samples when they arrive in host memory, and the staging of their Stokes
// products before the reorder (at most staging_cap; larger blocks run in
// channel passes through it) -- fits the caller's arena.
// Jobs admitted together are fused into one persistent-kernel launch
// (lbf_beamform_batch) on the next stream of the pool, so blocks arriving
// while others run overlap on the device.  Weights stay cached on the device
// per observation id and are evicted least-recently-used when the arena is
// short.  Completion is observed through HIP events by the scheduler thread.
// Blocks of one stream (stream_id != 0) run in order; the samples of an
// integration period left incomplete at the end of a block stay in a per-stream
// tail buffer in the arena and are prepended to the stream's next block.
// (Section 4.1: the station stream is cut into short blocks; Section 7:
// independent observations run in parallel while resources allow; Section 4.7:
// a bounded buffer that refuses work rather than stalling the pipeline.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
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

#include "../../include/lbf.h"
#include "lbf_internal.h"
#include "lbf_launch.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit sub-allocator over [0, size) of the caller's arena.
class Arena {
  public:
    void reset(uint64_t size) {
        free_.clear();
        size_ = size;
        if (size) free_[0] = size;
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, base = it->first;
                free_.erase(it);
                if (rest) free_[base + bytes] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    uint64_t used() const { return used_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0, used_ = 0;
};

int bytes_per_complex(int xt) { return xt == LBF_CI8 ? 2 : xt == LBF_CI16 ? 4 : 8; }
// bytes of one time sample of one station and channel: the X and Y polarisations
int sample_bytes(int xt) { return 2 * bytes_per_complex(xt); }
int weight_bytes(int ct) { return ct == LBF_F32 ? 8 : 4; }

struct WeightEntry {
    uint64_t off = 0, bytes = 0;   // weights + geometry scratch, one allocation
    int S = 0, B = 0, C = 0, ctype = 0;
    int refs = 0;
    uint64_t last_use = 0;
    hipEvent_t ready = nullptr;
};

struct JobRec {
    uint64_t ticket = 0;
    lbf_job job;
    std::vector<double> pos, dir, freq, delay;   // delay: [S] residual delays, or empty
    double ref[3];
    bool has_ref = false;
    lbf_job_status st;
    uint64_t x_off = 0, x_bytes = 0;   // staging of host samples
    bool staged = false;
    uint64_t wkey = 0;
    bool new_weights = false;
    // stream blocks: samples carried in from the tail, left in it afterwards,
    // and run now (carry_in + T - carry_out, a whole number of periods)
    int carry_in = 0, carry_out = 0, t_eff = 0;
    uint64_t cat_off = 0, cat_bytes = 0;   // [S][C][t_eff]: carried samples, then x
    bool has_cat = false;
    uint64_t stage_off = 0, stage_bytes = 0;   // Stokes staging (0 bytes: none needed)
    struct StreamState* ss = nullptr;
};

// A stream's tail: the samples [S][C][carried] of its incomplete integration
// period, pitch t_int - 1 samples.  Host bookkeeping (carried, pending) follows
// admission order; the device copies that read and write the tail are ordered
// by `ev`, recorded after each block's copies.
struct StreamState {
    int S = 0, C = 0, xtype = 0, t_int = 0;
    int carried = 0;              // samples in the tail after the last admitted block
    int pending = 0;              // admitted blocks not yet done
    bool broken = false;          // a block failed: later blocks fail too
    uint64_t tail_off = 0, tail_bytes = 0;
    hipEvent_t ev = nullptr;
    bool ev_valid = false;
};

struct Launch {
    std::vector<uint64_t> tickets;
    hipEvent_t done = nullptr;
    int stream = 0;
};

}  // namespace

struct lbf_server {
    lbf_server_cfg cfg;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<JobRec>> jobs;
    std::map<uint64_t, WeightEntry> wcache;   // key: obs_id * 4 + ctype
    std::unordered_map<uint64_t, StreamState> sstate;
    std::vector<Launch> inflight;
    int inflight_jobs = 0;
    Arena arena;
    uint64_t next_ticket = 1, use_clock = 0;
    bool stop = false;
    std::thread worker;
    std::string err;
};

namespace {

int validate_job(const lbf_job* j) {
    using lbf::set_error;
    if (!j) return set_error(LBF_E_INVAL, "lbf_server_submit: job is NULL");
    if (j->S < 1 || j->B < 1 || j->C < 1 || j->T < 1)
        return set_error(LBF_E_INVAL, "lbf_server_submit: sizes must be >= 1");
    if (!j->station_xyz || !j->beam_dir || !j->freq_hz || !j->x || !j->d_out)
        return set_error(LBF_E_INVAL, "lbf_server_submit: NULL pointer in job");
    if (j->xtype < LBF_CI8 || j->xtype > LBF_CF32) return set_error(LBF_E_INVAL, "lbf_server_submit: unknown xtype");
    if (j->ctype < LBF_F32 || j->ctype > LBF_BF16) return set_error(LBF_E_INVAL, "lbf_server_submit: unknown ctype");
    if (j->product != LBF_VOLTAGES && j->product != LBF_STOKES_I && j->product != LBF_STOKES_IQUV)
        return set_error(LBF_E_INVAL, "lbf_server_submit: unknown product");
    if (j->t_int < 1 || j->f_int < 1) return set_error(LBF_E_INVAL, "lbf_server_submit: t_int, f_int must be >= 1");
    if (j->stream_id != 0 && (j->product == LBF_VOLTAGES || j->x_on_host))
        return set_error(LBF_E_INVAL, "lbf_server_submit: stream blocks take Stokes products of device samples");
    if (j->product == LBF_VOLTAGES) {
        if (j->t_int != 1 || j->f_int != 1)
            return set_error(LBF_E_INVAL, "lbf_server_submit: voltages take t_int = f_int = 1");
    } else {
        if ((j->stream_id == 0 && j->T % j->t_int) || j->C % j->f_int)
            return set_error(LBF_E_INVAL, "lbf_server_submit: t_int must divide T and f_int must divide C");
        if (j->t_int & (j->t_int - 1))
            return set_error(LBF_E_UNSUPPORTED, "lbf_server_submit: t_int must be a power of two");
    }
    return LBF_OK;
}

uint64_t weights_alloc_bytes(const lbf_job& j) {
    return align_up((uint64_t)j.C * j.B * j.S * weight_bytes(j.ctype)) +
           align_up(sizeof(double) * ((uint64_t)j.S * 4 + (uint64_t)j.B * 3 + j.C));
}

uint64_t staging_bytes(const lbf_job& j) {
    return j.x_on_host ? (uint64_t)j.S * j.C * j.T * sample_bytes(j.xtype) : 0;
}

// samples [S][C][n] of a stream block
uint64_t stream_bytes(const lbf_job& j, int n) { return (uint64_t)j.S * j.C * n * sample_bytes(j.xtype); }

// the most a stream block can ever hold in the arena besides weights
uint64_t stream_max_bytes(const lbf_job& j) {
    if (!j.stream_id) return 0;
    return align_up(stream_bytes(j, j.T + j.t_int - 1)) + align_up(stream_bytes(j, j.t_int - 1));
}

// Stokes staging of a job: one channel's bytes for its longest block (a stream
// block runs up to T + t_int - 1 samples), and what admission reserves: all
// channels, or staging_cap when that is less.
uint64_t stage_cap(const lbf_server_cfg& c) { return c.staging_cap ? c.staging_cap : (256ull << 20); }

uint64_t stage_channel_bytes(const lbf_job& j) {
    lbf_block b;
    b.d_x = j.x; b.xtype = j.xtype;
    b.S = j.S; b.C = j.C;
    b.T = j.stream_id ? (j.T + j.t_int - 1) / j.t_int * j.t_int : j.T;
    b.d_w = j.x; b.ctype = j.ctype; b.B = j.B;
    b.product = j.product; b.t_int = j.t_int; b.f_int = j.f_int;
    b.d_out = j.d_out;
    return lbf::block_staging_channel_bytes(&b);
}

uint64_t stage_need(const lbf_server_cfg& c, const lbf_job& j) {
    const uint64_t per = stage_channel_bytes(j);
    if (per == 0) return 0;
    return std::min<uint64_t>(per * (uint64_t)j.C, stage_cap(c));
}

char* arena_ptr(lbf_server* s, uint64_t off) { return (char*)s->cfg.d_arena + off; }

enum { kAdmitWait = 0, kAdmitted = 1, kAdmitReject = 2 };

// Give a stream's tail back to the arena (no block of it may be pending).
void drop_tail(lbf_server* s, StreamState* ss) {
    if (ss->tail_bytes) s->arena.release(ss->tail_off, ss->tail_bytes);
    ss->tail_bytes = 0;
    if (ss->ev) (void)hipEventDestroy(ss->ev);
    ss->ev = nullptr;
    ss->ev_valid = false;
}

bool stream_shape_differs(const StreamState& ss, const lbf_job& j) {
    return ss.S != j.S || ss.C != j.C || ss.xtype != j.xtype || ss.t_int != j.t_int;
}

// Try to place a job's device state.  Called with the lock held.  Returns
// kAdmitWait when it must wait for memory (or for an in-use weight set), and
// kAdmitReject (with r->st.error set) when it can never run.
int try_admit(lbf_server* s, JobRec* r) {
    const lbf_job& j = r->job;
    // stream blocks: what is carried in, run, and carried out
    int cin = 0, cout = 0, teff = j.T;
    uint64_t need_cat = 0, need_tail = 0;
    StreamState* ss = nullptr;
    if (j.stream_id) {
        auto f = s->sstate.find(j.stream_id);
        if (f != s->sstate.end()) {
            ss = &f->second;
            if (ss->broken) {
                r->st.error = LBF_E_HIP;
                return kAdmitReject;
            }
            if (stream_shape_differs(*ss, j)) {   // the carried samples cannot continue: end the stream
                ss->broken = true;
                if (ss->pending == 0) drop_tail(s, ss);
                r->st.error = LBF_E_INVAL;
                return kAdmitReject;
            }
            cin = ss->carried;
        }
        cout = (cin + j.T) % j.t_int;
        teff = cin + j.T - cout;
        if (teff > 0 && (cin > 0 || cout > 0)) need_cat = stream_bytes(j, teff);
        if (cout > 0 && (!ss || ss->tail_bytes == 0)) need_tail = stream_bytes(j, j.t_int - 1);
    }
    const uint64_t key = j.obs_id * 4 + (uint64_t)j.ctype;
    auto it = s->wcache.find(key);
    bool hit = it != s->wcache.end() && it->second.S == j.S && it->second.B == j.B && it->second.C == j.C;
    if (it != s->wcache.end() && !hit && it->second.refs > 0) return kAdmitWait;   // same id, other shape, in use
    const uint64_t need[5] = {hit ? 0 : weights_alloc_bytes(j), staging_bytes(j), need_cat, need_tail,
                              stage_need(s->cfg, j)};
    uint64_t off[5] = {0, 0, 0, 0, 0};
    for (;;) {
        int k = 0;
        for (; k < 5; ++k)
            if (need[k] && !s->arena.alloc(need[k], &off[k])) break;
        if (k == 5) break;
        for (int i = 0; i < k; ++i)
            if (need[i]) s->arena.release(off[i], need[i]);
        // evict the least recently used idle weight set (never the one we need)
        auto victim = s->wcache.end();
        for (auto w = s->wcache.begin(); w != s->wcache.end(); ++w)
            if (w->second.refs == 0 && w->first != key &&
                (victim == s->wcache.end() || w->second.last_use < victim->second.last_use))
                victim = w;
        if (victim == s->wcache.end()) return kAdmitWait;
        (void)hipEventDestroy(victim->second.ready);
        s->arena.release(victim->second.off, victim->second.bytes);
        s->wcache.erase(victim);
    }
    if (!hit) {
        if (it != s->wcache.end()) {   // stale entry of another shape, idle
            (void)hipEventDestroy(it->second.ready);
            s->arena.release(it->second.off, it->second.bytes);
            s->wcache.erase(it);
        }
        WeightEntry e;
        e.off = off[0];
        e.bytes = need[0];
        e.S = j.S; e.B = j.B; e.C = j.C; e.ctype = j.ctype;
        (void)hipEventCreateWithFlags(&e.ready, hipEventDisableTiming);
        s->wcache[key] = e;
        r->new_weights = true;
    }
    WeightEntry& e = s->wcache[key];
    e.refs++;
    e.last_use = ++s->use_clock;
    r->wkey = key;
    if (need[1]) {
        r->x_off = off[1];
        r->x_bytes = need[1];
        r->staged = true;
    }
    if (need[4]) {
        r->stage_off = off[4];
        r->stage_bytes = need[4];
    }
    if (j.stream_id) {
        if (!ss) {
            ss = &s->sstate[j.stream_id];
            ss->S = j.S; ss->C = j.C; ss->xtype = j.xtype; ss->t_int = j.t_int;
        }
        if (need_tail) {
            ss->tail_off = off[3];
            ss->tail_bytes = need_tail;
        }
        ss->carried = cout;
        ss->pending++;
        r->ss = ss;
        r->carry_in = cin;
        r->carry_out = cout;
        if (need_cat) {
            r->cat_off = off[2];
            r->cat_bytes = need_cat;
            r->has_cat = true;
        }
    }
    r->t_eff = teff;
    r->st.periods = teff / j.t_int;
    return kAdmitted;
}

// Give back a finished (or failed) job's arena memory; a stream whose last
// admitted block is done and that carries nothing gives back its tail too.
void release_job(lbf_server* s, JobRec* r, bool failed) {
    if (r->staged) {
        s->arena.release(r->x_off, r->x_bytes);
        r->staged = false;
    }
    if (r->has_cat) {
        s->arena.release(r->cat_off, r->cat_bytes);
        r->has_cat = false;
    }
    if (r->stage_bytes) {
        s->arena.release(r->stage_off, r->stage_bytes);
        r->stage_bytes = 0;
    }
    if (StreamState* ss = r->ss) {
        r->ss = nullptr;
        if (failed) ss->broken = true;
        if (--ss->pending == 0 && (ss->carried == 0 || ss->broken)) {
            drop_tail(s, ss);
            if (!ss->broken) s->sstate.erase(r->job.stream_id);
        }
    }
    auto it = s->wcache.find(r->wkey);
    if (it != s->wcache.end() && it->second.refs > 0) it->second.refs--;
}

// Device copies of a stream block, ordered after the previous block's: the
// carried samples and the first teff - carry_in samples of x into the
// concatenation, then the last carry_out samples of x into the tail (or, when
// no period completes, all of x appended to the tail).
int stream_copies(lbf_server* s, JobRec* r, hipStream_t st) {
    const lbf_job& j = r->job;
    StreamState* ss = r->ss;
    if (!ss->ev && hipEventCreateWithFlags(&ss->ev, hipEventDisableTiming) != hipSuccess) return LBF_E_HIP;
    if (ss->ev_valid && hipStreamWaitEvent(st, ss->ev, 0) != hipSuccess) return LBF_E_HIP;
    const size_t bpc = sample_bytes(j.xtype), rows = (size_t)j.S * j.C;
    const size_t xp = (size_t)j.T * bpc, tp = (size_t)(j.t_int - 1) * bpc;
    const char* x = (const char*)j.x;
    char* tail = ss->tail_bytes ? arena_ptr(s, ss->tail_off) : nullptr;
    const int cin = r->carry_in, cout = r->carry_out, teff = r->t_eff;
    auto copy2d = [&](void* dst, size_t dp, const void* src, size_t sp, size_t w) {
        return w == 0 || hipMemcpy2DAsync(dst, dp, src, sp, w, rows, hipMemcpyDeviceToDevice, st) == hipSuccess;
    };
    bool ok = true;
    if (teff == 0) {
        ok = copy2d(tail + cin * bpc, tp, x, xp, xp);
    } else if (r->has_cat) {
        char* cat = arena_ptr(s, r->cat_off);
        const size_t cp = (size_t)teff * bpc;
        ok = copy2d(cat, cp, tail, tp, cin * bpc) &&
             copy2d(cat + cin * bpc, cp, x, xp, (size_t)(teff - cin) * bpc) &&
             copy2d(tail, tp, x + (size_t)(j.T - cout) * bpc, xp, cout * bpc);
    }
    if (!ok || hipEventRecord(ss->ev, st) != hipSuccess) return LBF_E_HIP;
    ss->ev_valid = true;
    return LBF_OK;
}

lbf_block block_of(lbf_server* s, JobRec* r) {
    const lbf_job& j = r->job;
    const WeightEntry& e = s->wcache[r->wkey];
    lbf_block b;
    b.d_x = r->staged ? (const void*)arena_ptr(s, r->x_off) : r->has_cat ? (const void*)arena_ptr(s, r->cat_off) : j.x;
    b.xtype = j.xtype;
    b.S = j.S; b.C = j.C; b.T = r->t_eff;
    b.d_w = arena_ptr(s, e.off);
    b.ctype = j.ctype;
    b.B = j.B;
    b.product = j.product;
    b.t_int = j.t_int;
    b.f_int = j.f_int;
    b.d_out = j.d_out;
    return b;
}

// Issue the work of a set of admitted jobs on one stream.  Called WITHOUT the
// lock; the JobRec objects and cache entries it touches are pinned by refs.
int issue(lbf_server* s, const std::vector<JobRec*>& rs, const std::vector<lbf_block>& blocks,
          const std::vector<WeightEntry>& went, hipStream_t st) {
    for (size_t i = 0; i < rs.size(); ++i) {
        JobRec* r = rs[i];
        const lbf_job& j = r->job;
        const WeightEntry& e = went[i];
        if (r->new_weights) {
            char* base = arena_ptr(s, e.off);
            double* geo = (double*)(base + align_up((uint64_t)j.C * j.B * j.S * weight_bytes(j.ctype)));
            double* dpos = geo;
            double* ddir = geo + (size_t)j.S * 3;
            double* dfreq = ddir + (size_t)j.B * 3;
            double* ddelay = dfreq + j.C;
            hipError_t he = hipMemcpyAsync(dpos, r->pos.data(), sizeof(double) * r->pos.size(), hipMemcpyHostToDevice, st);
            if (he == hipSuccess)
                he = hipMemcpyAsync(ddir, r->dir.data(), sizeof(double) * r->dir.size(), hipMemcpyHostToDevice, st);
            if (he == hipSuccess)
                he = hipMemcpyAsync(dfreq, r->freq.data(), sizeof(double) * r->freq.size(), hipMemcpyHostToDevice, st);
            if (he == hipSuccess && !r->delay.empty())
                he = hipMemcpyAsync(ddelay, r->delay.data(), sizeof(double) * r->delay.size(), hipMemcpyHostToDevice,
                                    st);
            if (he != hipSuccess) return LBF_E_HIP;
            int rc = lbf_compute_weights(dpos, j.S, ddir, j.B, r->has_ref ? r->ref : nullptr,
                                         r->delay.empty() ? nullptr : ddelay, dfreq, j.C, j.ctype, base, nullptr, st);
            if (rc) return rc;
            if (hipEventRecord(e.ready, st) != hipSuccess) return LBF_E_HIP;
        } else {
            if (hipStreamWaitEvent(st, e.ready, 0) != hipSuccess) return LBF_E_HIP;
        }
        if (r->staged) {
            if (hipMemcpyAsync(arena_ptr(s, r->x_off), j.x, r->x_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
                return LBF_E_HIP;
        }
        if (r->ss) {
            int rc = stream_copies(s, r, st);
            if (rc) return rc;
        }
    }
    if (blocks.empty()) return LBF_OK;
    // each block's Stokes staging is the slice its job reserved in the arena
    std::vector<void*> stage;
    std::vector<size_t> cap;
    for (JobRec* r : rs) {
        if (r->t_eff <= 0) continue;                  // as in the scheduler: no block for this job
        stage.push_back(r->stage_bytes ? (void*)arena_ptr(s, r->stage_off) : nullptr);
        cap.push_back((size_t)r->stage_bytes);
    }
    bool fused = blocks.size() > 1;
    for (const lbf_block& b : blocks)
        if (b.product == LBF_VOLTAGES || b.ctype == LBF_F32 || b.ctype != blocks[0].ctype) fused = false;
    if (fused) return lbf::run_batch(blocks.data(), (int)blocks.size(), stage.data(), cap.data(), st, "server");
    for (size_t i = 0; i < blocks.size(); ++i) {
        int rc = stage[i] ? lbf::run_block(&blocks[i], stage[i], cap[i], st, "server")
                          : lbf::run_block(&blocks[i], nullptr, 0, st, "server");
        if (rc) return rc;
    }
    return LBF_OK;
}

void scheduler(lbf_server* s) {
    (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // 1. completions
        for (size_t i = 0; i < s->inflight.size();) {
            Launch& L = s->inflight[i];
            hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) { ++i; continue; }
            const uint64_t t = now_ns();
            for (uint64_t tk : L.tickets) {
                auto it = s->jobs.find(tk);
                if (it == s->jobs.end()) continue;
                JobRec* r = it->second.get();
                r->st.state = q == hipSuccess ? LBF_JOB_DONE : LBF_JOB_FAILED;
                r->st.error = q == hipSuccess ? LBF_OK : LBF_E_HIP;
                r->st.t_done_ns = t;
                release_job(s, r, q != hipSuccess);
                s->inflight_jobs--;
            }
            (void)hipEventDestroy(L.done);
            s->inflight[i] = s->inflight.back();
            s->inflight.pop_back();
            s->cv_done.notify_all();
        }
        // 2. admission (arrival order) into one batch
        std::vector<JobRec*> batch;
        while (!s->queue.empty() && (int)batch.size() < s->cfg.max_batch &&
               s->inflight_jobs < s->cfg.max_inflight) {
            auto it = s->jobs.find(s->queue.front());
            if (it == s->jobs.end()) { s->queue.pop_front(); continue; }
            JobRec* r = it->second.get();
            const int a = try_admit(s, r);
            if (a == kAdmitWait) break;
            if (a == kAdmitReject) {   // a broken stream, or a block whose shape is not its stream's
                r->st.state = LBF_JOB_FAILED;
                r->st.t_done_ns = now_ns();
                s->queue.pop_front();
                s->cv_done.notify_all();
                continue;
            }
            r->st.state = LBF_JOB_ADMITTED;
            r->st.t_admit_ns = now_ns();
            s->queue.pop_front();
            s->inflight_jobs++;
            batch.push_back(r);
        }
        // 3. launch
        if (!batch.empty()) {
            std::vector<lbf_block> blocks;
            std::vector<WeightEntry> went;
            for (JobRec* r : batch) {
                if (r->t_eff > 0) blocks.push_back(block_of(s, r));   // a stream block may complete no period
                went.push_back(s->wcache[r->wkey]);
            }
            const int si = s->next_stream;
            s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
            hipStream_t st = s->streams[si];
            lk.unlock();
            const uint64_t t0 = now_ns();
            int rc = issue(s, batch, blocks, went, st);
            hipEvent_t ev = nullptr;
            if (rc == LBF_OK && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) rc = LBF_E_HIP;
            if (rc == LBF_OK && hipEventRecord(ev, st) != hipSuccess) rc = LBF_E_HIP;
            lk.lock();
            if (rc != LBF_OK) {
                // the stream may hold part of the batch: wait for it before
                // giving the memory back
                lk.unlock();
                (void)hipStreamSynchronize(st);
                lk.lock();
                if (ev) (void)hipEventDestroy(ev);
                for (JobRec* r : batch) {
                    r->st.state = LBF_JOB_FAILED;
                    r->st.error = rc;
                    r->st.t_done_ns = now_ns();
                    release_job(s, r, true);
                    s->inflight_jobs--;
                }
                // weights this batch was to compute are not valid: drop them
                for (JobRec* r : batch) {
                    if (!r->new_weights) continue;
                    auto it = s->wcache.find(r->wkey);
                    if (it == s->wcache.end() || it->second.refs > 0) continue;
                    (void)hipEventDestroy(it->second.ready);
                    s->arena.release(it->second.off, it->second.bytes);
                    s->wcache.erase(it);
                }
                s->cv_done.notify_all();
            } else {
                Launch L;
                L.done = ev;
                L.stream = si;
                for (JobRec* r : batch) {
                    r->st.state = LBF_JOB_RUNNING;
                    r->st.t_start_ns = t0;
                    r->st.batch_size = (int)batch.size();
                    L.tickets.push_back(r->ticket);
                }
                s->inflight.push_back(L);
            }
            continue;
        }
        if (s->stop && s->queue.empty() && s->inflight.empty()) break;
        if (s->inflight.empty()) s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

int lbf_server_create(const lbf_server_cfg* cfg, lbf_server** out) {
    using lbf::set_error;
    if (!cfg || !out) return set_error(LBF_E_INVAL, "lbf_server_create: NULL argument");
    if (!cfg->d_arena || cfg->arena_bytes == 0 || cfg->max_inflight < 1 || cfg->n_streams < 1 ||
        cfg->queue_capacity < 1 || cfg->max_batch < 1 || cfg->max_batch > LBF_MAX_BATCH || cfg->device < 0)
        return set_error(LBF_E_INVAL, "lbf_server_create: malformed configuration");
    std::unique_ptr<lbf_server> s(new lbf_server());
    s->cfg = *cfg;
    s->arena.reset(cfg->arena_bytes);
    if (hipSetDevice(cfg->device) != hipSuccess) return set_error(LBF_E_HIP, "lbf_server_create: hipSetDevice failed");
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            return set_error(LBF_E_HIP, "lbf_server_create: stream creation failed");
        }
        s->streams.push_back(st);
    }
    lbf_server* raw = s.release();
    raw->worker = std::thread(scheduler, raw);
    *out = raw;
    return LBF_OK;
}

int lbf_server_submit(lbf_server* s, const lbf_job* job, uint64_t* ticket) {
    using lbf::set_error;
    if (!s || !ticket) return set_error(LBF_E_INVAL, "lbf_server_submit: NULL argument");
    int rc = validate_job(job);
    if (rc) return rc;
    // a channel pass holds whole groups of f_int channels (channel integration)
    const uint64_t group = job->product == LBF_VOLTAGES ? 1 : (uint64_t)job->f_int;
    if (stage_channel_bytes(*job) * group > stage_cap(s->cfg))
        return set_error(LBF_E_NOMEM, "lbf_server_submit: the Stokes staging of one channel (of f_int channels "
                         "with channel integration) exceeds staging_cap");
    if (weights_alloc_bytes(*job) + align_up(staging_bytes(*job)) + stream_max_bytes(*job) +
            align_up(stage_need(s->cfg, *job)) > s->cfg.arena_bytes)
        return set_error(LBF_E_NOMEM, "lbf_server_submit: job footprint exceeds the arena");
    std::unique_ptr<JobRec> r(new JobRec());
    r->job = *job;
    r->pos.assign(job->station_xyz, job->station_xyz + (size_t)job->S * 3);
    r->dir.assign(job->beam_dir, job->beam_dir + (size_t)job->B * 3);
    r->freq.assign(job->freq_hz, job->freq_hz + job->C);
    if (job->station_delay) r->delay.assign(job->station_delay, job->station_delay + job->S);
    if (job->ref_dir) {
        memcpy(r->ref, job->ref_dir, sizeof(r->ref));
        r->has_ref = true;
    }
    r->job.station_xyz = nullptr;
    r->job.beam_dir = nullptr;
    r->job.freq_hz = nullptr;
    r->job.ref_dir = nullptr;
    r->job.station_delay = nullptr;
    memset(&r->st, 0, sizeof(r->st));
    r->st.state = LBF_JOB_QUEUED;
    r->st.t_submit_ns = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_error(LBF_E_INVAL, "lbf_server_submit: server is shutting down");
    if ((int)s->queue.size() >= s->cfg.queue_capacity) return set_error(LBF_E_BUSY, "lbf_server_submit: queue full");
    if (job->stream_id) {
        auto f = s->sstate.find(job->stream_id);
        if (f != s->sstate.end() && f->second.broken)
            return set_error(LBF_E_HIP, "lbf_server_submit: an earlier block of this stream failed");
        if (f != s->sstate.end() && stream_shape_differs(f->second, *job))
            return set_error(LBF_E_INVAL, "lbf_server_submit: S, C, xtype and t_int must stay those of the stream");
    }
    const uint64_t t = s->next_ticket++;
    r->ticket = t;
    s->jobs[t] = std::move(r);
    s->queue.push_back(t);
    *ticket = t;
    s->cv_work.notify_one();
    return LBF_OK;
}

int lbf_server_poll(lbf_server* s, uint64_t ticket, lbf_job_status* st) {
    if (!s || !st) return LBF_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return lbf::set_error(LBF_E_NOTFOUND, "lbf_server_poll: unknown ticket");
    *st = it->second->st;
    return LBF_OK;
}

int lbf_server_wait(lbf_server* s, uint64_t ticket, int timeout_ms, lbf_job_status* st) {
    if (!s || !st) return LBF_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    for (;;) {
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) return LBF_E_NOTFOUND;
        const int state = it->second->st.state;
        if (state == LBF_JOB_DONE || state == LBF_JOB_FAILED) {
            *st = it->second->st;
            return LBF_OK;
        }
        if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            auto it2 = s->jobs.find(ticket);
            if (it2 == s->jobs.end()) return LBF_E_NOTFOUND;
            *st = it2->second->st;
            return (st->state == LBF_JOB_DONE || st->state == LBF_JOB_FAILED) ? LBF_OK : LBF_E_BUSY;
        }
    }
}

int lbf_server_release(lbf_server* s, uint64_t ticket) {
    if (!s) return LBF_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return LBF_E_NOTFOUND;
    const int state = it->second->st.state;
    if (state != LBF_JOB_DONE && state != LBF_JOB_FAILED) return LBF_E_BUSY;
    s->jobs.erase(it);
    return LBF_OK;
}

int lbf_server_destroy(lbf_server* s) {
    if (!s) return LBF_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->wcache) (void)hipEventDestroy(kv.second.ready);
    for (auto& kv : s->sstate)
        if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    delete s;
    return LBF_OK;
}

}  // extern "C"
