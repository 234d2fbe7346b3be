// Continuous-batching engine: many XC integrations (one per SCF iteration of
// many molecules) share the device. Requests are admitted by device-memory
// footprint; an admitted request's grid, weights, batches and screening
// lists stay on the device across its iterations (grid reuse, Sec. 2.3.1),
// and so, when the budget allows, do its collocation matrices Phi^j (they
// depend on the grid and the basis only); every step co-batches the pending
// grid batches of all in-flight integrations into the same launches (Alg. 4
// over a mixed batch set). Grids of newly admitted requests are built by a
// builder thread on a stream of its own, so building never holds up the
// steps of the requests already running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "xc_internal.hpp"

namespace xc {

struct Integration {
    long long ticket = 0;
    long long req = 0;
    const double* P = nullptr;
    double* V = nullptr;
    double* EN = nullptr;
    long long next_batch = 0;
    bool started = false;
    bool launched_finish = false;
    hipEvent_t done = nullptr;
    int error = XC_OK;          // its request could not be admitted
};

struct Request {
    long long id = 0;
    xc_context* ctx = nullptr;
    int functional = XC_GGA_PBE;
    int precision = XC_FP64;
    size_t est_bytes = 0;
    size_t bytes = 0;
    bool building = false;      // handed to the builder thread
    bool est_charged = false;   // est_bytes counted in the engine's used bytes
    std::atomic<bool> built{false};  // set by the builder thread when done
    int build_rc = XC_OK;       // its result (valid once built)
    bool admitted = false;
    bool released = false;
    int error = XC_OK;          // set when the request cannot be admitted
    std::string error_msg;
    std::deque<Integration*> queued;
    Integration* active = nullptr;
    // collocation matrices kept across the request's integrations
    bool cache = false;
    bool phi_ready = false;     // the first integration has written them
    DevBuf phi_store;
    std::vector<long long> phi_offs;  // per batch, doubles from phi_store
};

}  // namespace xc

struct xc_engine {
    hipStream_t stream = nullptr;
    int device = 0;
    size_t budget = 0;
    size_t wave_bytes = 0;
    size_t used = 0;
    bool cache_phi = false;
    xc::DevBuf scratch, d_wb, d_gpre, d_spre, d_wpre, d_reqs, d_tmap;
    std::map<long long, xc::Request*> reqs;
    std::deque<long long> waiting;
    std::map<long long, xc::Integration*> tickets;
    long long next_req = 1, next_ticket = 1;
    long long steps = 0, batches_launched = 0, completed = 0, colloc_batches = 0;
    xc::PhaseTimer timer;
    // builder thread
    hipStream_t build_stream = nullptr;
    std::thread builder;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<xc::Request*> build_q;
    bool stop = false;
};

namespace xc {

int build_grid(xc_context* c);

// The builder thread: builds the grids of admitted requests, one at a time,
// on its own stream (the build synchronises that stream, not the engine's).
static void builder_main(xc_engine* e) {
    (void)hipSetDevice(e->device);
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(e->mu);
            e->cv.wait(lk, [&] { return e->stop || !e->build_q.empty(); });
            if (e->stop) return;
            r = e->build_q.front();
            e->build_q.pop_front();
        }
        xc_context* c = r->ctx;
        c->stream = e->build_stream;
        int rc = build_grid(c);
        if (rc == XC_OK) {
            release_build_temporaries(c);
            for (const WaveBatch& w : c->h_wb)
                if (batch_scratch_bytes(w) > e->wave_bytes) {
                    rc = fail(XC_ERR_NOMEM, "a batch is larger than the engine's wave scratch");
                    break;
                }
        }
        if (rc == XC_OK && r->precision == XC_MIXED_BF16) {
            rc = dev_reserve(c->pdig, 8 * (size_t)c->nbf * c->nbf);
            if (rc == XC_OK) rc = dev_reserve(c->pscale, 8 * (size_t)c->nbf);
        }
        if (rc == XC_OK) {
            hipError_t st = hipStreamSynchronize(e->build_stream);
            if (st != hipSuccess) rc = hip_fail(st, "hipStreamSynchronize(build stream)");
        }
        if (rc != XC_OK) r->error_msg = xc_last_error();
        c->stream = e->stream;
        r->build_rc = rc;
        r->built.store(true, std::memory_order_release);
    }
}

// Hand waiting requests whose estimated footprint fits to the builder, and
// finish the admission of those whose grids are built: the estimate is
// replaced by the actual bytes, and the Phi store is added when caching is
// on and the budget allows it.
static int admit(xc_engine* e) {
    for (auto it = e->waiting.begin(); it != e->waiting.end();) {
        Request* r = e->reqs[*it];
        if (r->released) {
            it = e->waiting.erase(it);
            continue;
        }
        if (!r->building) {
            if (e->used + r->est_bytes > e->budget) {
                ++it;
                continue;
            }
            r->building = true;
            r->est_charged = true;
            e->used += r->est_bytes;
            {
                std::lock_guard<std::mutex> lk(e->mu);
                e->build_q.push_back(r);
            }
            e->cv.notify_one();
            ++it;
            continue;
        }
        if (!r->built.load(std::memory_order_acquire)) {
            ++it;
            continue;
        }
        xc_context* c = r->ctx;
        e->used -= std::min(e->used, r->est_bytes);
        r->est_charged = false;
        int rc = r->build_rc;
        if (rc != XC_OK) {
            // the request can never run: it leaves the queue with its device
            // memory released, and its integrations report the error
            r->error = rc;
            for (Integration* in : r->queued) in->error = rc;
            r->queued.clear();
            xc_context_destroy(c);
            r->ctx = nullptr;
            it = e->waiting.erase(it);
            return fail(rc, r->error_msg);
        }
        r->bytes = device_bytes(c);
        if (e->cache_phi) {
            size_t store = 0;
            r->phi_offs.clear();
            for (const WaveBatch& w : c->h_wb) {
                r->phi_offs.push_back((long long)(store / 8));
                store += batch_phi_bytes(w);
            }
            if (e->used + r->bytes + store <= e->budget &&
                dev_reserve(r->phi_store, std::max<size_t>(store, 8)) == XC_OK) {
                r->cache = true;
                r->bytes += r->phi_store.cap;
            } else {
                (void)hipGetLastError();
                r->phi_offs.clear();
            }
        }
        e->used += r->bytes;
        r->admitted = true;
        it = e->waiting.erase(it);
    }
    return XC_OK;
}

static void destroy_request(xc_engine* e, Request* r) {
    if (r->ctx) {
        xc_context_destroy(r->ctx);
        r->ctx = nullptr;
    }
    dev_release(r->phi_store);
    if (r->admitted) e->used -= std::min(e->used, r->bytes);
    r->admitted = false;
}

struct Group {
    std::vector<WaveBatch> wb;
    std::vector<int> gpre{0}, spre{0}, wpre{0};
    std::vector<ReqDev> rd;
    std::map<Integration*, int> slot;
    int gemm = 0, syr = 0, wide = 0;
    double s2 = 0.0, s1 = 0.0;   // sum n_b^2 n_g and sum n_b n_g of the group's batches
    bool sph = false;   // some request of the group has spherical shells
};

static int engine_step(xc_engine* e, int* launched) {
    *launched = 0;
    XC_TRY(admit(e));
    // activate the next queued integration of every admitted request
    std::vector<Integration*> act;
    for (auto& kv : e->reqs) {
        Request* r = kv.second;
        if (!r->admitted) continue;
        if (!r->active && !r->queued.empty()) {
            r->active = r->queued.front();
            r->queued.pop_front();
        }
        if (r->active && !r->active->launched_finish) act.push_back(r->active);
    }
    std::sort(act.begin(), act.end(),
              [](const Integration* a, const Integration* b) { return a->ticket < b->ticket; });
    if (act.empty()) return XC_OK;
    // zero V (and cut P into digits in split-BF16 mode) of integrations that
    // start now
    for (Integration* in : act) {
        if (in->started) continue;
        const Request* r = e->reqs[in->req];
        const int nbf = r->ctx->nbf;
        const long long nn = (long long)nbf * nbf;
        XC_TRY(launch_fill(e->stream, in->V, nn, 0.0));
        if (r->precision == XC_MIXED_BF16)
            XC_TRY(launch_p_digits(e->stream, in->P, nbf, (unsigned long long*)r->ctx->pdig.p,
                                   (double*)r->ctx->pscale.p));
        in->started = true;
    }
    // round-robin: one batch of each in-flight integration at a time until the
    // wave scratch is full or every integration is exhausted
    std::map<int, Group> groups;  // key: precision * 2 + gga
    size_t used = 0;
    bool progress = true;
    while (progress) {
        progress = false;
        for (Integration* in : act) {
            Request* r = e->reqs[in->req];
            xc_context* c = r->ctx;
            if (in->next_batch >= c->n_batches) continue;
            WaveBatch w = c->h_wb[in->next_batch];
            const size_t bytes = r->cache ? batch_zpart_bytes(w) : batch_scratch_bytes(w);
            if (used + bytes > e->wave_bytes) continue;
            const int key = r->precision * 2 + (r->functional == XC_GGA_PBE ? 1 : 0);
            Group& g = groups[key];
            g.sph = g.sph || c->any_pure;
            auto sl = g.slot.find(in);
            int req_slot;
            if (sl == g.slot.end()) {
                req_slot = (int)g.rd.size();
                g.slot[in] = req_slot;
                ReqDev rd = make_req(c, in->P, in->V);
                rd.phi_base = r->cache ? (char*)r->phi_store.p : nullptr;
                g.rd.push_back(rd);
            } else {
                req_slot = sl->second;
            }
            const long long slab = (long long)w.nbp * w.ngp;
            if (r->cache) {
                w.phi_off = r->phi_offs[in->next_batch];
                w.z_off = (long long)(used / 8);
                w.flags = r->phi_ready ? kSkipColloc : 0;
            } else {
                w.phi_off = (long long)(used / 8);
                w.z_off = w.phi_off + (long long)(batch_phi_bytes(w) / 8);
                w.flags = 0;
            }
            w.part_off = w.z_off + slab;
            if (!(w.flags & kSkipColloc)) e->colloc_batches += 1;
            w.req = req_slot;
            used += bytes;
            const int gt = w.nmt * (w.ngp / kTile);
            const int st = w.nmt * (w.nmt + 1) / 2;
            const int pt = batch_wide_tiles(w);
            g.wb.push_back(w);
            g.gpre.push_back(g.gpre.back() + gt);
            g.spre.push_back(g.spre.back() + st);
            g.wpre.push_back(g.wpre.back() + pt);
            g.gemm += gt;
            g.syr += st;
            g.wide += pt;
            g.s1 += (double)w.nb * w.ng;
            g.s2 += (double)w.nb * w.nb * w.ng;
            in->next_batch += 1;
            *launched += 1;
            progress = true;
        }
    }
    // upload the descriptors of every group (one array each, groups back to back)
    std::vector<WaveBatch> all_wb;
    std::vector<int> all_g, all_s, all_p;
    std::vector<ReqDev> all_rd;
    struct Off { size_t wb, pre, rd; };
    std::map<int, Off> offs;
    for (auto& kv : groups) {
        Group& g = kv.second;
        Off o{all_wb.size(), all_g.size(), all_rd.size()};
        for (WaveBatch& w : g.wb) w.req += (int)o.rd;
        offs[kv.first] = o;
        all_wb.insert(all_wb.end(), g.wb.begin(), g.wb.end());
        all_g.insert(all_g.end(), g.gpre.begin(), g.gpre.end());
        all_s.insert(all_s.end(), g.spre.begin(), g.spre.end());
        all_p.insert(all_p.end(), g.wpre.begin(), g.wpre.end());
        all_rd.insert(all_rd.end(), g.rd.begin(), g.rd.end());
    }
    if (!all_wb.empty()) {
        // growing a descriptor buffer frees the old one: let earlier steps that
        // read it finish first
        int max_tiles = 1;
        for (const auto& kv : groups) max_tiles = std::max({max_tiles, kv.second.gemm, kv.second.syr});
        const size_t need[6] = {sizeof(WaveBatch) * all_wb.size(), sizeof(int) * all_g.size(),
                                sizeof(int) * all_s.size(), sizeof(ReqDev) * all_rd.size(),
                                2 * sizeof(int) * (size_t)max_tiles, sizeof(int) * all_p.size()};
        const DevBuf* bufs[6] = {&e->d_wb,   &e->d_gpre, &e->d_spre,
                                 &e->d_reqs, &e->d_tmap, &e->d_wpre};
        for (int q = 0; q < 6; ++q) {
            if (bufs[q]->cap < need[q]) {
                XC_HIP(hipStreamSynchronize(e->stream));
                break;
            }
        }
        XC_TRY(dev_reserve(e->d_wb, 2 * need[0]));
        XC_TRY(dev_reserve(e->d_gpre, 2 * need[1]));
        XC_TRY(dev_reserve(e->d_spre, 2 * need[2]));
        XC_TRY(dev_reserve(e->d_reqs, 2 * need[3]));
        XC_TRY(dev_reserve(e->d_tmap, 2 * need[4]));
        XC_TRY(dev_reserve(e->d_wpre, 2 * need[5]));
        XC_TRY(upload(e->d_wb, all_wb.data(), sizeof(WaveBatch) * all_wb.size(), e->stream));
        XC_TRY(upload(e->d_gpre, all_g.data(), sizeof(int) * all_g.size(), e->stream));
        XC_TRY(upload(e->d_spre, all_s.data(), sizeof(int) * all_s.size(), e->stream));
        XC_TRY(upload(e->d_wpre, all_p.data(), sizeof(int) * all_p.size(), e->stream));
        XC_TRY(upload(e->d_reqs, all_rd.data(), sizeof(ReqDev) * all_rd.size(), e->stream));
        for (auto& kv : groups) {
            const Group& g = kv.second;
            const Off& o = offs[kv.first];
            const int precision = kv.first / 2;
            const bool gga = kv.first & 1;
            XC_TRY(launch_wave(&e->timer, e->stream, gga, precision,
                               (const WaveBatch*)e->d_wb.p + o.wb,
                               (const int*)e->d_gpre.p + o.pre,
                               (const int*)e->d_spre.p + o.pre,
                               (const int*)e->d_wpre.p + o.pre, (int)g.wb.size(), g.gemm,
                               g.syr, g.wide, g.s2 >= kWideNb * g.s1,
                               (const ReqDev*)e->d_reqs.p, (char*)e->scratch.p,
                               (int*)e->d_tmap.p, true, g.sph));
        }
        e->batches_launched += *launched;
    }
    // finish integrations whose last batch has been launched
    for (Integration* in : act) {
        Request* r = e->reqs[in->req];
        xc_context* c = r->ctx;
        if (in->next_batch < c->n_batches || in->launched_finish) continue;
        XC_TRY(launch_finish(&e->timer, e->stream, in->V, c->nbf, (const double*)c->epart.p,
                             (const double*)c->npart.p, c->n_batches, in->EN));
        XC_HIP(hipEventCreateWithFlags(&in->done, hipEventDisableTiming));
        XC_HIP(hipEventRecord(in->done, e->stream));
        in->launched_finish = true;
        r->active = nullptr;
        // every batch's Phi is in the store now (later launches are ordered
        // after these on the stream)
        if (r->cache) r->phi_ready = true;
    }
    e->steps += 1;
    return XC_OK;
}

}  // namespace xc

using namespace xc;

extern "C" {

int xc_engine_create(const xc_engine_opts* opts, xc_engine** out) {
    if (!out) return fail(XC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    xc_engine* e = new (std::nothrow) xc_engine();
    if (!e) return fail(XC_ERR_NOMEM, "host allocation failed");
    e->stream = opts ? (hipStream_t)opts->stream : nullptr;
    size_t fr = 0, tot = 0;
    hipError_t st = hipMemGetInfo(&fr, &tot);
    if (st != hipSuccess) {
        delete e;
        return hip_fail(st, "hipMemGetInfo");
    }
    e->wave_bytes = (opts && opts->wave_bytes) ? opts->wave_bytes
                                               : std::min<size_t>(fr / 8, (size_t)8 << 30);
    e->budget = (opts && opts->hbm_budget) ? opts->hbm_budget : fr / 2;
    e->cache_phi = opts && opts->cache_phi;
    st = hipGetDevice(&e->device);
    if (st != hipSuccess) {
        delete e;
        return hip_fail(st, "hipGetDevice");
    }
    int rc = dev_reserve(e->scratch, e->wave_bytes);
    if (rc != XC_OK) {
        delete e;
        return rc;
    }
    // default priority, like every stream of the library
    st = hipStreamCreateWithFlags(&e->build_stream, hipStreamNonBlocking);
    if (st != hipSuccess) {
        dev_release(e->scratch);
        delete e;
        return hip_fail(st, "hipStreamCreateWithFlags");
    }
    try {
        e->builder = std::thread(builder_main, e);
    } catch (...) {
        (void)hipStreamDestroy(e->build_stream);
        dev_release(e->scratch);
        delete e;
        return fail(XC_ERR_NOMEM, "could not start the grid builder thread");
    }
    *out = e;
    return XC_OK;
}

int xc_engine_add_request(xc_engine* e, const xc_molecule* mol, const xc_basis* basis,
                          const xc_grid_spec* grid, int functional, int precision,
                          long long* req_id) {
    if (!e || !req_id) return fail(XC_ERR_INVALID_ARG, "null engine or output");
    if (functional != XC_LDA_SVWN5 && functional != XC_GGA_PBE)
        return fail(XC_ERR_UNSUPPORTED, "unknown functional");
    if (precision != XC_FP64 && precision != XC_MIXED_FP32 && precision != XC_MIXED_FP32_V &&
        precision != XC_MIXED_BF16)
        return fail(XC_ERR_UNSUPPORTED, "precision not available");
    xc_device_opts o{e->stream, 0};
    xc_context* c = nullptr;
    XC_TRY(xc_context_create(mol, basis, grid, &o, &c));
    Request* r = new (std::nothrow) Request();
    if (!r) {
        xc_context_destroy(c);
        return fail(XC_ERR_NOMEM, "host allocation failed");
    }
    r->id = e->next_req++;
    r->ctx = c;
    r->functional = functional;
    r->precision = precision;
    r->est_bytes = estimate_build_bytes(c);
    if (precision == XC_MIXED_BF16) r->est_bytes += 8 * (size_t)c->nbf * (c->nbf + 1);
    if (r->est_bytes > e->budget) {
        xc_context_destroy(c);
        delete r;
        return fail(XC_ERR_NOMEM, "request larger than the engine's memory budget");
    }
    e->reqs[r->id] = r;
    e->waiting.push_back(r->id);
    *req_id = r->id;
    return XC_OK;
}

int xc_engine_submit(xc_engine* e, long long req_id, const double* d_P, double* d_V,
                     double* d_EN, long long* ticket) {
    if (!e || !ticket || !d_P || !d_V || !d_EN)
        return fail(XC_ERR_INVALID_ARG, "null engine, buffer or output");
    auto it = e->reqs.find(req_id);
    if (it == e->reqs.end() || it->second->released)
        return fail(XC_ERR_INVALID_ARG, "unknown or released request");
    if (it->second->error != XC_OK)
        return fail(it->second->error, "request could not be admitted: " + it->second->error_msg);
    Integration* in = new (std::nothrow) Integration();
    if (!in) return fail(XC_ERR_NOMEM, "host allocation failed");
    in->ticket = e->next_ticket++;
    in->req = req_id;
    in->P = d_P;
    in->V = d_V;
    in->EN = d_EN;
    it->second->queued.push_back(in);
    e->tickets[in->ticket] = in;
    *ticket = in->ticket;
    return XC_OK;
}

int xc_engine_step(xc_engine* e, int* n_batches) {
    if (!e) return fail(XC_ERR_INVALID_ARG, "null engine");
    int dummy = 0;
    return engine_step(e, n_batches ? n_batches : &dummy);
}

int xc_engine_poll(xc_engine* e, long long ticket, int* done) {
    if (!e || !done) return fail(XC_ERR_INVALID_ARG, "null engine or output");
    auto it = e->tickets.find(ticket);
    if (it == e->tickets.end()) return fail(XC_ERR_INVALID_ARG, "unknown ticket");
    Integration* in = it->second;
    *done = 0;
    if (in->error != XC_OK) {
        const int rc = in->error;
        e->tickets.erase(it);
        delete in;
        return fail(rc, "the ticket's request could not be admitted");
    }
    if (!in->done) return XC_OK;
    hipError_t q = hipEventQuery(in->done);
    if (q == hipErrorNotReady) return XC_OK;
    if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    *done = 1;
    (void)hipEventDestroy(in->done);
    e->tickets.erase(it);
    delete in;
    e->completed += 1;
    return XC_OK;
}

int xc_engine_release(xc_engine* e, long long req_id) {
    if (!e) return fail(XC_ERR_INVALID_ARG, "null engine");
    auto it = e->reqs.find(req_id);
    if (it == e->reqs.end()) return fail(XC_ERR_INVALID_ARG, "unknown request");
    Request* r = it->second;
    if (r->active || !r->queued.empty())
        return fail(XC_ERR_BUSY, "request still has integrations in flight");
    // a grid being built is the builder thread's until it is done
    if (r->building)
        while (!r->built.load(std::memory_order_acquire)) std::this_thread::yield();
    if (r->est_charged) {
        e->used -= std::min(e->used, r->est_bytes);
        r->est_charged = false;
    }
    e->waiting.erase(std::remove(e->waiting.begin(), e->waiting.end(), req_id),
                     e->waiting.end());
    r->released = true;
    destroy_request(e, r);
    e->reqs.erase(it);
    delete r;
    return XC_OK;
}

int xc_engine_stats(xc_engine* e, xc_engine_info* s) {
    if (!e || !s) return fail(XC_ERR_INVALID_ARG, "null engine or stats");
    std::memset(s, 0, sizeof(*s));
    for (auto& kv : e->reqs) {
        if (kv.second->admitted) s->admitted += 1;
        else s->waiting += 1;
        if (kv.second->active) s->in_flight += 1;
    }
    s->bytes_used = e->used;
    s->budget = e->budget;
    s->wave_bytes = e->wave_bytes;
    s->steps = e->steps;
    s->batches_launched = e->batches_launched;
    s->completed = e->completed;
    s->colloc_batches = e->colloc_batches;
    for (auto& kv : e->reqs) s->phi_cached += kv.second->cache ? 1 : 0;
    return XC_OK;
}

int xc_engine_destroy(xc_engine* e) {
    if (!e) return XC_OK;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->stop = true;
    }
    e->cv.notify_all();
    if (e->builder.joinable()) e->builder.join();
    (void)hipStreamSynchronize(e->build_stream);
    (void)hipStreamDestroy(e->build_stream);
    (void)hipStreamSynchronize(e->stream);
    for (auto& kv : e->tickets) {
        if (kv.second->done) (void)hipEventDestroy(kv.second->done);
        delete kv.second;
    }
    for (auto& kv : e->reqs) {
        destroy_request(e, kv.second);
        delete kv.second;
    }
    DevBuf* bufs[] = {&e->scratch, &e->d_wb,   &e->d_gpre, &e->d_spre,
                      &e->d_wpre,  &e->d_reqs, &e->d_tmap};
    for (DevBuf* b : bufs) dev_release(*b);
    delete e;
    return XC_OK;
}

}  // extern "C"
