// Request server: keeps the index on the device and aligns requests (batches of
// reads of mixed length) as they arrive, with continuous batching.
//
// The HBM budget is split into S slots. Each slot owns a HIP stream, a device
// arena (reads, lengths, outputs, align workspace) and pinned host staging, and is
// driven by its own host thread. A slot that is free takes every waiting request
// that fits its capacity (same d_max, FIFO order), copies them in, runs the
// batched align on its stream, copies the outputs out and completes the requests.
// Requests that arrive while other slots are busy are admitted by the next slot
// that frees up, and the slots' work overlaps on the device. A read's output does
// not depend on the other reads in its batch, so a request's result is the same
// alone and in the mix.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/snapgpu.h"
#include "snap_internal.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t ticket;
    int64_t n;
    int64_t bases;
    int32_t d_max;
    std::vector<uint8_t> reads;
    std::vector<int32_t> lengths;
    std::vector<int64_t> pos;
    std::vector<int8_t> strand;
    std::vector<int32_t> dist, second;
    std::vector<int8_t> call;
    double t_submit = 0, t_start = 0, t_done = 0;
    int status = SNAP_EAGAIN;
};

struct Slot {
    hipStream_t stream = nullptr;
    char *dev = nullptr;          // slot's slice of the device arena
    size_t dev_bytes = 0;
    char *host = nullptr;         // pinned staging
    size_t host_bytes = 0;
    std::thread th;
};

}  // namespace

struct snap_server {
    const snap_index *ix;
    snap_params params;
    snap_server_config cfg;
    snap_tuning tuning;
    bool has_tuning = false;
    int device = 0;
    char *arena = nullptr;
    size_t ws_bytes = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> waiting;
    std::unordered_map<uint64_t, Req *> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::atomic<int64_t> batches{0}, completed{0}, busy{0}, failed{0};
    int64_t submitted = 0;
};

namespace {

// Device layout of one slot: reads, lengths, the five outputs, the align workspace.
struct SlotLayout {
    size_t reads, lengths, pos, strand, dist, second, call, ws, total;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

SlotLayout slot_layout(int64_t R, int64_t B, size_t ws) {
    SlotLayout l{};
    size_t o = 0;
    l.reads = o; o = a256(o + (size_t)B);
    l.lengths = o; o = a256(o + 4 * (size_t)R);
    l.pos = o; o = a256(o + 8 * (size_t)R);
    l.strand = o; o = a256(o + (size_t)R);
    l.dist = o; o = a256(o + 4 * (size_t)R);
    l.second = o; o = a256(o + 4 * (size_t)R);
    l.call = o; o = a256(o + (size_t)R);
    l.ws = o; o = a256(o + ws);
    l.total = o;
    return l;
}

// Host staging: reads and lengths in, outputs out.
size_t host_bytes(int64_t R, int64_t B) { return a256((size_t)B) + a256(4 * (size_t)R) + a256(18 * (size_t)R); }

void run_slot(snap_server *s, int k) {
    Slot &sl = s->slots[k];
    (void)hipSetDevice(s->device);
    const SlotLayout L = slot_layout(s->cfg.batch_reads, s->cfg.batch_bases, s->ws_bytes);
    for (;;) {
        std::vector<Req *> batch;
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv.wait(g, [&] { return s->stop || !s->waiting.empty(); });
            if (s->waiting.empty() && s->stop) return;
            // admit every waiting request that fits this slot, oldest first, same d_max
            int64_t nr = 0, nb = 0;
            const int32_t dm = s->waiting.front()->d_max;
            for (auto it = s->waiting.begin(); it != s->waiting.end();) {
                Req *r = *it;
                if (r->d_max == dm && nr + r->n <= s->cfg.batch_reads && nb + r->bases <= s->cfg.batch_bases) {
                    nr += r->n;
                    nb += r->bases;
                    batch.push_back(r);
                    it = s->waiting.erase(it);
                } else {
                    ++it;
                }
            }
        }
        s->busy++;
        const double t0 = now_s();
        int64_t nr = 0, nb = 0;
        char *h = sl.host;
        uint8_t *h_reads = (uint8_t *)h;
        int32_t *h_len = (int32_t *)(h + a256((size_t)s->cfg.batch_bases));
        char *h_out = (char *)h_len + a256(4 * (size_t)s->cfg.batch_reads);
        for (Req *r : batch) {
            r->t_start = t0;
            std::memcpy(h_reads + nb, r->reads.data(), (size_t)r->bases);
            std::memcpy(h_len + nr, r->lengths.data(), 4 * (size_t)r->n);
            nr += r->n;
            nb += r->bases;
        }
        char *d = sl.dev;
        int rc = SNAP_OK;
        if (hipMemcpyAsync(d + L.reads, h_reads, (size_t)nb, hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
            hipMemcpyAsync(d + L.lengths, h_len, 4 * (size_t)nr, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            rc = SNAP_EDEVICE;
        if (rc == SNAP_OK)
            rc = snap_align_batched(s->ix, (const uint8_t *)(d + L.reads), (const int32_t *)(d + L.lengths), nr,
                                    batch.front()->d_max, &s->params, s->has_tuning ? &s->tuning : nullptr,
                                    (int64_t *)(d + L.pos), (int8_t *)(d + L.strand), (int32_t *)(d + L.dist),
                                    (int32_t *)(d + L.second), (int8_t *)(d + L.call), d + L.ws, s->ws_bytes,
                                    sl.stream);
        // outputs back: pos 8, strand 1, dist 4, second 4, call 1 bytes per read
        int64_t *h_pos = (int64_t *)h_out;
        int32_t *h_dist = (int32_t *)(h_pos + nr);
        int32_t *h_second = h_dist + nr;
        int8_t *h_strand = (int8_t *)(h_second + nr);
        int8_t *h_call = h_strand + nr;
        if (rc == SNAP_OK &&
            (hipMemcpyAsync(h_pos, d + L.pos, 8 * (size_t)nr, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
             hipMemcpyAsync(h_dist, d + L.dist, 4 * (size_t)nr, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
             hipMemcpyAsync(h_second, d + L.second, 4 * (size_t)nr, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
             hipMemcpyAsync(h_strand, d + L.strand, (size_t)nr, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
             hipMemcpyAsync(h_call, d + L.call, (size_t)nr, hipMemcpyDeviceToHost, sl.stream) != hipSuccess))
            rc = SNAP_EDEVICE;
        // on every path, success or not: the slot's staging buffers are reused by its next
        // batch, so nothing queued on its stream (the copies in, a partly queued alignment)
        // may still be running when they are overwritten
        if (hipStreamSynchronize(sl.stream) != hipSuccess && rc == SNAP_OK) rc = SNAP_EDEVICE;
        const double t1 = now_s();
        int64_t o = 0;
        {
            std::lock_guard<std::mutex> g(s->mu);
            for (Req *r : batch) {
                if (rc == SNAP_OK) {
                    r->pos.assign(h_pos + o, h_pos + o + r->n);
                    r->strand.assign(h_strand + o, h_strand + o + r->n);
                    r->dist.assign(h_dist + o, h_dist + o + r->n);
                    r->second.assign(h_second + o, h_second + o + r->n);
                    r->call.assign(h_call + o, h_call + o + r->n);
                }
                o += r->n;
                r->t_done = t1;
                r->status = rc;
                std::vector<uint8_t>().swap(r->reads);
                std::vector<int32_t>().swap(r->lengths);
            }
        }
        s->batches++;
        s->completed += (int64_t)batch.size();
        if (rc != SNAP_OK) s->failed += (int64_t)batch.size();
        s->busy--;
        s->cv.notify_all();
    }
}

}  // namespace

extern "C" snap_server_config snap_server_default_config(void) {
    snap_server_config c;
    std::memset(&c, 0, sizeof(c));
    c.hbm_budget = 8ull << 30;
    c.slots = 4;
    c.max_waiting = 4096;
    c.batch_reads = 1 << 18;
    c.batch_bases = 256ll << 20;
    c.max_len = 16384;
    c.d_max = 8;
    return c;
}

extern "C" int snap_server_create(const snap_index *ix, const snap_params *p, const snap_server_config *cfg,
                                  const snap_tuning *tuning, snap_server **out) {
    if (!out) return SNAP_EINVAL;
    *out = nullptr;
    if (!ix || !p || !cfg || cfg->slots < 1 || cfg->max_waiting < 1 || cfg->batch_reads < 1 ||
        cfg->batch_bases < 1 || cfg->max_len < 1 || cfg->d_max < 0 || cfg->hbm_budget == 0)
        return SNAP_EINVAL;
    const size_t ws = snap_align_workspace_bytes(ix, cfg->batch_reads, cfg->batch_bases, cfg->max_len, cfg->d_max, p);
    if (ws == 0) return SNAP_EINVAL;
    snap_server *s = new (std::nothrow) snap_server();
    if (!s) return SNAP_ENOMEM;
    s->ix = ix;
    s->params = *p;
    s->cfg = *cfg;
    if (tuning) { s->tuning = *tuning; s->has_tuning = true; }
    s->ws_bytes = ws * 2;   // room for larger passes than the minimum
    const SlotLayout L = slot_layout(cfg->batch_reads, cfg->batch_bases, s->ws_bytes);
    const int nslots = (int)std::min<uint64_t>((uint64_t)cfg->slots, cfg->hbm_budget / L.total);
    if (nslots < 1) { delete s; return SNAP_ENOMEM; }
    s->cfg.slots = nslots;
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return SNAP_EDEVICE; }
    if (hipMalloc((void **)&s->arena, L.total * (size_t)nslots) != hipSuccess) { delete s; return SNAP_ENOMEM; }
    s->slots.resize(nslots);
    const size_t hb = host_bytes(cfg->batch_reads, cfg->batch_bases);
    int rc = SNAP_OK;
    for (int k = 0; k < nslots; k++) {
        Slot &sl = s->slots[k];
        sl.dev = s->arena + L.total * (size_t)k;
        sl.dev_bytes = L.total;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) { rc = SNAP_EDEVICE; break; }
        if (hipHostMalloc((void **)&sl.host, hb, hipHostMallocDefault) != hipSuccess) { rc = SNAP_ENOMEM; break; }
        sl.host_bytes = hb;
    }
    if (rc != SNAP_OK) {
        snap_server_destroy(s);
        return rc;
    }
    for (int k = 0; k < nslots; k++) s->slots[k].th = std::thread(run_slot, s, k);
    *out = s;
    return SNAP_OK;
}

extern "C" int snap_server_submit(snap_server *s, const uint8_t *reads, const int32_t *lengths, int64_t n,
                                  int32_t d_max, uint64_t *ticket) {
    if (!s || !ticket || n < 0 || (n > 0 && (!reads || !lengths)) || d_max != s->cfg.d_max) return SNAP_EINVAL;
    int64_t bases = 0;
    for (int64_t i = 0; i < n; i++) {
        if (lengths[i] < 0 || lengths[i] > s->cfg.max_len) return SNAP_EINVAL;
        bases += lengths[i];
    }
    if (n > s->cfg.batch_reads || bases > s->cfg.batch_bases) return SNAP_EINVAL;
    Req *r = new (std::nothrow) Req();
    if (!r) return SNAP_ENOMEM;
    r->n = n;
    r->bases = bases;
    r->d_max = d_max;
    r->reads.assign(reads, reads + bases);
    r->lengths.assign(lengths, lengths + n);
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) { delete r; return SNAP_EINVAL; }
        if ((int64_t)s->waiting.size() >= s->cfg.max_waiting) { delete r; return SNAP_EBUSY; }
        r->ticket = s->next_ticket++;
        r->t_submit = now_s();
        s->reqs[r->ticket] = r;
        s->waiting.push_back(r);
        s->submitted++;
        *ticket = r->ticket;
    }
    s->cv.notify_all();
    return SNAP_OK;
}

extern "C" int snap_server_poll(snap_server *s, uint64_t ticket, snap_result *out) {
    if (!s || !out) return SNAP_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SNAP_EINVAL;
    Req *r = it->second;
    if (r->status == SNAP_EAGAIN) return SNAP_EAGAIN;
    std::memset(out, 0, sizeof(*out));
    out->n = r->n;
    out->status = r->status;
    out->pos = r->pos.data();
    out->strand = r->strand.data();
    out->dist = r->dist.data();
    out->second = r->second.data();
    out->call = r->call.data();
    out->t_submit = r->t_submit;
    out->t_start = r->t_start;
    out->t_done = r->t_done;
    return SNAP_OK;
}

extern "C" int snap_server_release(snap_server *s, uint64_t ticket) {
    if (!s) return SNAP_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SNAP_EINVAL;
    if (it->second->status == SNAP_EAGAIN) return SNAP_EAGAIN;
    delete it->second;
    s->reqs.erase(it);
    return SNAP_OK;
}

extern "C" int snap_server_stats(snap_server *s, snap_server_stats_t *out) {
    if (!s || !out) return SNAP_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->slots = s->cfg.slots;
    out->submitted = s->submitted;
    out->completed = s->completed.load();
    out->failed = s->failed.load();
    out->batches = s->batches.load();
    out->waiting = (int64_t)s->waiting.size();
    out->busy_slots = s->busy.load();
    out->slot_device_bytes = s->slots.empty() ? 0 : s->slots[0].dev_bytes;
    return SNAP_OK;
}

extern "C" int snap_server_destroy(snap_server *s) {
    if (!s) return SNAP_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (auto &sl : s->slots)
        if (sl.th.joinable()) sl.th.join();   // slots finish every admitted and waiting request first
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.host) (void)hipHostFree(sl.host);
    }
    if (s->arena) (void)hipFree(s->arena);
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
    return SNAP_OK;
}
