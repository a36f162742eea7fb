// Request server: assemble-and-solve requests of different meshes and
// horizons, admitted by estimated HBM footprint into slots that run
// concurrently on their own HIP streams (continuous batching: a request that
// arrives while others run starts as soon as a slot and pool memory are free).
//
// Each slot is a worker thread with its own stream and a context that draws
// device memory from the server's pool.  A request runs the whole path on its
// slot: plan (ball query, classification, pattern), numeric assembly, CG, and
// the copy of the solution to host memory.  Every kernel's result depends on
// the request's inputs only, so a request gives bitwise the same solution
// alone and in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "common.hpp"
#include "runtime.hpp"

using namespace nlfem;

namespace {

using Clock = std::chrono::steady_clock;

double seconds_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
}

struct Request {
    uint64_t ticket = 0;
    // owned host copies of the inputs
    int64_t V = 0, K = 0;
    std::vector<double> coords, f, g;
    std::vector<int32_t> tets;
    std::vector<uint8_t> vfree, region, mask;
    nlfem_params prm{};
    double rtol = 1e-10;
    int32_t max_iter = 0;
    // scheduling
    size_t est = 0;      // admission estimate (pool bytes)
    size_t est_raw = 0;  // the geometric estimate before calibration
    int est_class = 0;   // calibration class: quarter-octave of est_raw
    bool measured = false;  // est comes from a measured need (re-queue), not the model
    int skipped = 0;
    Clock::time_point t_arrival, t_admit, t_plan, t_assemble, t_done;
    double queue_s = 0, plan_s = 0, assemble_s = 0, solve_s = 0;
    // results
    nlfem_request_info info{};
    std::string err;
    std::vector<double> x;
    std::vector<int32_t> f2v;
};

// Host-side footprint estimate of one request (bytes of pool memory at the
// peak of its run): pair and candidate lists from the horizon ball over the
// mesh's mean tet density, ball vertex sets and CSR rows from the vertex
// density, plus the fixed per-tet and per-vertex arrays.
size_t estimate_footprint(const Request& r) {
    const int64_t V = r.V, K = r.K;
    if (K == 0) return (size_t)1 << 20;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < V; ++v)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], r.coords[3 * v + d]);
            hi[d] = std::max(hi[d], r.coords[3 * v + d]);
        }
    double ext = 0.0;
    int64_t n_outer = 0;
    for (int64_t e = 0; e < K; ++e) {
        double a[3] = {1e300, 1e300, 1e300}, b[3] = {-1e300, -1e300, -1e300};
        bool has_free = false;
        for (int j = 0; j < 4; ++j) {
            const int32_t v = r.tets[4 * e + j];
            if (v < 0 || v >= V) continue;
            has_free |= r.vfree[v] != 0;
            for (int d = 0; d < 3; ++d) {
                a[d] = std::min(a[d], r.coords[3 * v + d]);
                b[d] = std::max(b[d], r.coords[3 * v + d]);
            }
        }
        for (int d = 0; d < 3; ++d) ext = std::max(ext, b[d] - a[d]);
        const bool omega = r.region.empty() ? has_free : r.region[e] != 0;
        if (omega && (r.mask.empty() || r.mask[e])) ++n_outer;
    }
    int64_t nf = 0;
    for (int64_t v = 0; v < V; ++v) nf += r.vfree[v] ? 1 : 0;
    const double vol = std::max((hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]), 1e-300);
    const double dt = (double)K / vol, dv = (double)V / vol;
    const double pi43 = 4.18879020478639;
    const double d = r.prm.delta;
    auto ball = [&](double rad) { return pi43 * rad * rad * rad; };
    const double ppo = std::min((double)K, dt * ball(d + ext));                   // pairs per outer tet
    const double cpo = std::min((double)K, dt * std::pow(2.0 * (d + 2.0 * ext), 3));  // candidates
    const double vpo = std::min((double)V, dv * ball(d + 2.0 * ext));             // |Ve|
    const double row = std::min((double)V, dv * ball(d + 3.0 * ext));             // columns per row
    const double P = n_outer * ppo, C = n_outer * cpo, VT = n_outer * vpo, nnz = nf * row;
    const double mesh = V * 40.0 + K * 420.0;
    const double classify = C * 6.0 + P * 12.0 + n_outer * 64.0;
    // the element-keyed sample table (8 bytes per sample and element) stays with the plan
    const bool table = r.prm.keying == NLFEM_KEY_ELEMENT && r.prm.strategy == NLFEM_FULLCAPS &&
                       r.prm.cap_sampling != NLFEM_CAPS_OUTSIDE_UI;
    const double stab = table ? (double)K * 8.0 * (double)sample_table_stride(r.prm.mc_samples) : 0.0;
    const double retained = P * 6.0 + VT * 44.0 + n_outer * 200.0 + nnz * 20.0 + nf * 64.0 + stab;
    // the CSR pattern keeps each row's columns between its two passes: half
    // the row's hash set (a power of two of at least 4 |Ve| slots)
    const double rowcap = std::max(512.0, std::exp2(std::ceil(std::log2(4.0 * std::max(vpo, 1.0)))));
    // the local vertex sets pass through a hand-off buffer of a power of two
    // of at least half the pairs per outer tet, per outer tet (when that
    // stays within 2 GiB), before the CSR pattern's row buffer exists
    const double vstride = std::max(64.0, std::exp2(std::ceil(std::log2(std::max(ppo * 0.5, 1.0)))));
    const double vbuf = n_outer * vstride * 4.0 <= 2147483648.0 ? n_outer * vstride * 4.0 : 0.0;
    const double pattern = retained + VT * 24.0 + std::max((double)nf * (rowcap / 2.0) * 4.0, vbuf);
    const double numeric = retained + nnz * 12.0 + nf * 48.0;
    const double est = (mesh + std::max(classify, std::max(pattern, numeric))) * 1.25 + (double)(8 << 20);
    return (size_t)std::min(est, 1e18);
}

}  // namespace

struct nlfem_server {
    int device = 0;
    Pool pool;
    struct Slot {
        std::thread th;
        nlfem_ctx* ctx = nullptr;
        hipStream_t stream = nullptr;
        size_t reserved = 0;
    };
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    // calibration of the footprint model: per class of raw estimate, the
    // largest measured peak / raw estimate of a finished request
    std::map<int, double> ratio;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    bool stopping = false;
    size_t reserved = 0;
    int running = 0, max_running = 0;
    int64_t n_done = 0, n_failed = 0;
    std::string err;
};

namespace {

// Admission estimate: the geometric model scaled by the largest peak / model
// ratio measured so far on requests of the same class (raw estimates within a
// quarter octave), with a 15 % margin; the model alone until a request of the
// class has finished, and never above it (an underestimate that runs out of
// pool memory is re-queued with its measured need).
constexpr double kEstMargin = 1.15;

int est_class_of(size_t est_raw) { return (int)std::floor(4.0 * std::log2((double)std::max<size_t>(est_raw, 1))); }

void calibrate(nlfem_server* s, Request* r) {
    if (r->measured) return;
    const auto it = s->ratio.find(r->est_class);
    double f = 1.0;
    if (it != s->ratio.end()) f = std::min(1.0, it->second * kEstMargin);
    r->est = std::min((size_t)((double)r->est_raw * f), s->pool.size);
    r->info.est_bytes = r->est;
}

// picks the next request that fits (first fit in arrival order); a head that
// has been passed over 16 times blocks the others until it fits
Request* pick(nlfem_server* s) {
    for (size_t i = 0; i < s->queue.size(); ++i) {
        Request* r = s->queue[i];
        calibrate(s, r);
        if (s->reserved + r->est <= s->pool.size) {
            s->queue.erase(s->queue.begin() + (long)i);
            return r;
        }
        if (i == 0 && ++r->skipped > 16) return nullptr;
    }
    return nullptr;
}

// runs one request on the slot's context; returns its status
nlfem_status run_request(nlfem_server* s, nlfem_ctx* c, Request* r) {
    nlfem_mesh m{r->V, r->K, r->coords.data(), r->tets.data(), r->vfree.data(),
                 r->region.empty() ? nullptr : r->region.data(), 0};
    nlfem_params p = r->prm;
    p.outer_mask = r->mask.empty() ? nullptr : r->mask.data();
    nlfem_plan* pl = nullptr;
    std::vector<void*> bufs;
    auto cleanup = [&]() {
        hipStreamSynchronize(c->stream);
        for (void* b : bufs) dfree(c, b);
        if (pl) nlfem_plan_destroy(pl);
        drain_pending(c);
    };
    auto take = [&](size_t bytes) {
        void* b = dalloc(c, bytes);
        if (b) bufs.push_back(b);
        return b;
    };
    nlfem_status st = nlfem_plan_create(c, &m, &p, &pl);
    if (st != NLFEM_OK) {
        r->err = c->err;
        pl = nullptr;
        cleanup();
        return st;
    }
    r->t_plan = Clock::now();
    int64_t nf = 0, nff = 0, nfc = 0;
    nlfem_plan_info(pl, &nf, &nff, &nfc, r->info.pair_counts, nullptr);
    r->info.n_free = nf;
    r->info.nnz_ff = nff;
    r->info.nnz_fc = nfc;
    int64_t* rp = (int64_t*)take((size_t)(nf + 1) * 8);
    int32_t* ci = (int32_t*)take((size_t)(nff + 1) * 4);
    double* va = (double*)take((size_t)(nff + 1) * 8);
    double* rhs = (double*)take((size_t)(nf + 1) * 8);
    int32_t* f2v = (int32_t*)take((size_t)(nf + 1) * 4);
    double* x = (double*)take((size_t)(nf + 1) * 8);
    double* fd = r->f.empty() ? nullptr : (double*)take(r->f.size() * 8);
    double* gd = r->g.empty() ? nullptr : (double*)take(r->g.size() * 8);
    if (!rp || !ci || !va || !rhs || !f2v || !x || (!r->f.empty() && !fd) || (!r->g.empty() && !gd)) {
        r->err = c->err;
        cleanup();
        return NLFEM_E_OOM;
    }
    if (fd) hipMemcpyAsync(fd, r->f.data(), r->f.size() * 8, hipMemcpyHostToDevice, c->stream);
    if (gd) hipMemcpyAsync(gd, r->g.data(), r->g.size() * 8, hipMemcpyHostToDevice, c->stream);
    st = nlfem_assemble(pl, fd, gd, rp, ci, va, nullptr, nullptr, nullptr, rhs, f2v);
    if (st == NLFEM_OK && launch_fill_zero_f64(x, nf, c->stream) != hipSuccess) st = NLFEM_E_DEVICE;
    if (st == NLFEM_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = NLFEM_E_DEVICE;
    if (st != NLFEM_OK) {
        r->err = c->err;
        cleanup();
        return st;
    }
    r->t_assemble = Clock::now();
    int32_t it = 0;
    double rr = 0.0;
    const int32_t max_iter = r->max_iter > 0 ? r->max_iter : (int32_t)std::min<int64_t>(10 * nf + 100, 1 << 30);
    st = nlfem_cg(c, nf, rp, ci, va, rhs, x, r->rtol, max_iter, &it, &rr);
    r->info.cg_iters = it;
    r->info.cg_rel_residual = rr;
    if (st != NLFEM_OK && st != NLFEM_E_NOT_CONVERGED) {
        r->err = c->err;
        cleanup();
        return st;
    }
    r->x.resize((size_t)nf);
    r->f2v.resize((size_t)nf);
    if (nf) {
        hipMemcpyAsync(r->x.data(), x, (size_t)nf * 8, hipMemcpyDeviceToHost, c->stream);
        hipMemcpyAsync(r->f2v.data(), f2v, (size_t)nf * 4, hipMemcpyDeviceToHost, c->stream);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        r->err = "copy of the solution failed";
        cleanup();
        return NLFEM_E_DEVICE;
    }
    if (st == NLFEM_E_NOT_CONVERGED) r->err = "CG did not converge";
    cleanup();
    return st;
}

void worker(nlfem_server* s, int slot_id) {
    hipSetDevice(s->device);
    nlfem_server::Slot& slot = s->slots[slot_id];
    while (true) {
        Request* r = nullptr;
        int others = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stopping || (r = pick(s)) != nullptr; });
            if (!r) return;  // stopping
            s->reserved += r->est;
            slot.reserved = r->est;
            others = s->running;
            ++s->running;
            s->max_running = std::max(s->max_running, s->running);
            r->info.state = 1;
            r->info.attempts += 1;
            r->t_admit = Clock::now();
        }
        slot.ctx->peak = slot.ctx->live;
        slot.ctx->err.clear();
        const nlfem_status st = run_request(s, slot.ctx, r);
        const Clock::time_point t_end = Clock::now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->reserved -= slot.reserved;
            slot.reserved = 0;
            --s->running;
            r->info.peak_bytes = std::max(r->info.peak_bytes, slot.ctx->peak);
            const bool oom = st == NLFEM_E_OOM;
            if (oom && !(others == 0 && r->est >= s->pool.size) && r->info.attempts < 6) {
                // re-queue at the front with the measured need (at most the whole pool: then it runs alone)
                const size_t need = std::max<size_t>(2 * r->est, slot.ctx->peak + slot.ctx->peak / 2);
                r->est = std::min(need, s->pool.size);
                r->info.est_bytes = r->est;
                r->measured = true;
                r->info.state = 0;
                r->skipped = 0;
                s->queue.push_front(r);
            } else {
                r->t_done = t_end;
                r->info.status = st;
                r->info.state = (st == NLFEM_OK) ? 2 : 3;
                r->info.queue_s = seconds_between(r->t_arrival, r->t_admit);
                if (st == NLFEM_OK || st == NLFEM_E_NOT_CONVERGED) {
                    r->info.plan_s = seconds_between(r->t_admit, r->t_plan);
                    r->info.assemble_s = seconds_between(r->t_plan, r->t_assemble);
                    r->info.solve_s = seconds_between(r->t_assemble, t_end);
                }
                r->info.latency_s = seconds_between(r->t_arrival, t_end);
                if (st == NLFEM_OK && r->est_raw > 0) {
                    double& q = s->ratio[r->est_class];
                    q = std::max(q, (double)r->info.peak_bytes / (double)r->est_raw);
                }
                if (st == NLFEM_OK) ++s->n_done;
                else {
                    ++s->n_failed;
                    s->err = "request " + std::to_string(r->ticket) + ": " + r->err;
                }
            }
        }
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
}

void server_stop(nlfem_server* s) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto& sl : s->slots)
        if (sl.th.joinable()) sl.th.join();
    for (auto& sl : s->slots) {
        if (sl.ctx) nlfem_destroy(sl.ctx);
        if (sl.stream) hipStreamDestroy(sl.stream);
    }
    s->slots.clear();
    s->pool.destroy();
}

}  // namespace

extern "C" {

nlfem_status nlfem_server_create(int device, int32_t n_slots, size_t pool_bytes, nlfem_server** out) {
    if (!out || n_slots < 1 || n_slots > 64) return NLFEM_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        hipGetLastError();
        return NLFEM_E_DEVICE;
    }
    if (device < 0 || device >= n) return NLFEM_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return NLFEM_E_DEVICE;
    if (pool_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return NLFEM_E_DEVICE;
        pool_bytes = fr / 2;
    }
    nlfem_server* s = new nlfem_server();
    s->device = device;
    if (!s->pool.init(pool_bytes)) {
        delete s;
        return NLFEM_E_OOM;
    }
    s->slots.resize((size_t)n_slots);
    for (auto& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            nlfem_create(&sl.ctx, device, sl.stream, 0) != NLFEM_OK) {
            server_stop(s);
            delete s;
            return NLFEM_E_DEVICE;
        }
        sl.ctx->pool = &s->pool;
    }
    for (int i = 0; i < n_slots; ++i) s->slots[i].th = std::thread(worker, s, i);
    *out = s;
    return NLFEM_OK;
}

nlfem_status nlfem_server_submit(nlfem_server* s, const nlfem_mesh* mesh, const nlfem_params* prm,
                                 const double* f_qp, const double* g_nodal, const nlfem_solve_params* solve,
                                 uint64_t* ticket) {
    if (!s || !mesh || !prm || !ticket) return NLFEM_E_INVALID_ARG;
    if (mesh->mem_kind != 0) return NLFEM_E_INVALID_ARG;
    if (mesh->n_vertices < 0 || mesh->n_tets < 0) return NLFEM_E_INVALID_ARG;
    if (mesh->n_tets > 0 && (!mesh->coords || !mesh->tets || !mesh->vertex_free)) return NLFEM_E_INVALID_ARG;
    if (!(prm->delta > 0.0) || prm->mc_samples < 1 || prm->mc_samples > NLFEM_MAX_MC_SAMPLES)
        return NLFEM_E_INVALID_ARG;
    if (prm->strategy < NLFEM_FULLCAPS || prm->strategy > NLFEM_BARYCENTER) return NLFEM_E_INVALID_ARG;
    if (prm->cap_sampling != NLFEM_CAPS_WHOLE_ELEMENT && prm->cap_sampling != NLFEM_CAPS_OUTSIDE_UI)
        return NLFEM_E_INVALID_ARG;
    std::unique_ptr<Request> r(new Request());
    r->t_arrival = Clock::now();
    r->V = mesh->n_vertices;
    r->K = mesh->n_tets;
    r->coords.assign(mesh->coords, mesh->coords + 3 * r->V);
    r->tets.assign(mesh->tets, mesh->tets + 4 * r->K);
    r->vfree.assign(mesh->vertex_free, mesh->vertex_free + r->V);
    if (mesh->tet_region) r->region.assign(mesh->tet_region, mesh->tet_region + r->K);
    if (prm->outer_mask) r->mask.assign(prm->outer_mask, prm->outer_mask + r->K);
    if (f_qp) r->f.assign(f_qp, f_qp + 4 * r->K);
    if (g_nodal) r->g.assign(g_nodal, g_nodal + r->V);
    r->prm = *prm;
    r->prm.outer_mask = nullptr;
    if (solve) {
        r->rtol = solve->rtol;
        r->max_iter = solve->max_iter;
    }
    r->est_raw = estimate_footprint(*r);
    r->est_class = est_class_of(r->est_raw);
    r->est = std::min(r->est_raw, s->pool.size);
    r->info.est_bytes = r->est;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        *ticket = r->ticket;
        s->queue.push_back(r.get());
        s->reqs.emplace(r->ticket, std::move(r));
    }
    s->cv_work.notify_all();
    return NLFEM_OK;
}

nlfem_status nlfem_server_poll(nlfem_server* s, uint64_t ticket, nlfem_request_info* info) {
    if (!s || !info) return NLFEM_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return NLFEM_E_INVALID_ARG;
    *info = it->second->info;
    return NLFEM_OK;
}

nlfem_status nlfem_server_wait(nlfem_server* s, uint64_t ticket, double timeout_s, nlfem_request_info* info) {
    if (!s) return NLFEM_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return NLFEM_E_INVALID_ARG;
    Request* r = it->second.get();
    auto done = [&] { return r->info.state >= 2; };
    if (timeout_s < 0) s->cv_done.wait(lk, done);
    else s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    if (info) *info = r->info;
    return NLFEM_OK;
}

nlfem_status nlfem_server_take(nlfem_server* s, uint64_t ticket, double* x, int32_t* free_to_vertex) {
    if (!s) return NLFEM_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second->info.state < 2) return NLFEM_E_INVALID_ARG;
    Request* r = it->second.get();
    if (x && !r->x.empty()) std::copy(r->x.begin(), r->x.end(), x);
    if (free_to_vertex && !r->f2v.empty()) std::copy(r->f2v.begin(), r->f2v.end(), free_to_vertex);
    s->reqs.erase(it);
    return NLFEM_OK;
}

nlfem_status nlfem_server_stats(nlfem_server* s, nlfem_server_counters* st) {
    if (!s || !st) return NLFEM_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    st->queued = (int64_t)s->queue.size();
    st->running = s->running;
    st->done = s->n_done;
    st->failed = s->n_failed;
    st->max_running = s->max_running;
    st->n_slots = (int32_t)s->slots.size();
    st->pool_bytes = s->pool.size;
    {
        std::lock_guard<std::mutex> g(s->pool.mu);
        st->pool_used = s->pool.used;
        st->pool_peak = s->pool.peak;
    }
    return NLFEM_OK;
}

const char* nlfem_server_last_error(nlfem_server* s) { return s ? s->err.c_str() : "null server"; }

nlfem_status nlfem_server_destroy(nlfem_server* s) {
    if (!s) return NLFEM_E_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->queue.clear();  // queued requests are dropped; running ones finish
    }
    server_stop(s);
    delete s;
    return NLFEM_OK;
}

}  // extern "C"
