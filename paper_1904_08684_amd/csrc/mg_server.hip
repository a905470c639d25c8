// Solve server: many mixed-precision multigrid solves in flight on one GPU,
// continuously batched.
//
// Memory.  The caller hands the server one device arena.  Its head holds
// the per-hierarchy I/O pointer table, the per-hierarchy norm results and
// the launch tables; the rest is managed first-fit in 256-byte granules.
// Each admitted request gets a resident level hierarchy (a context laid out
// in its own arena block plus the device-resident op program of one
// refinement step).  Idle hierarchies stay resident for reuse by requests of
// the same shape; a request that needs memory evicts idle ones, least
// recently used first.  Admission is FIFO: the queue head is admitted when a
// slot is free and its footprint fits.
//
// Execution.  Requests advance in rounds.  A round runs, for every request
// in flight, one FP64 refinement step (residual with norm, power-of-two
// scaling, one single-precision V-cycle, update); a newly admitted request
// first loads its right-hand side and takes its initial residual in the
// same round.  The programs of all requests are merged by position: launch
// k of the round is one persistent batched kernel running op k of every
// request, whatever its level, size or dimension.  One device-to-host copy
// per round brings back every request's residual norm; converged requests
// unpack their solution to the caller's buffer and free their slot.
//
// Each request's arithmetic is the same whatever else is in flight: the
// same device functions run on its own hierarchy with per-request tilings
// and reductions.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_runtime.h"

namespace mg {
namespace {

constexpr size_t kGranule = 256;
constexpr int kMaxProgram = 1024;      // ops per request per round, upper bound
size_t gran(size_t v) { return (v + kGranule - 1) / kGranule * kGranule; }

// First-fit allocator over byte offsets [0, cap); adjacent free blocks merge.
class Arena {
  public:
    size_t cap = 0, used = 0, peak = 0;
    void init(size_t c) {
        cap = c;
        free_.clear();
        if (c) free_[0] = c;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = gran(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used += bytes;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = gran(bytes);
        used -= bytes;
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

  private:
    std::map<size_t, size_t> free_;
};

struct Key {
    int dim, n, smoother, nu1, nu2, post_order;
    double omega;
    bool operator==(const Key& o) const {
        return dim == o.dim && n == o.n && smoother == o.smoother && nu1 == o.nu1 && nu2 == o.nu2 &&
               post_order == o.post_order && omega == o.omega;
    }
};

struct Hier {
    Key key;
    size_t off = 0, bytes = 0, ctx_bytes = 0;
    Ctx* ctx = nullptr;
    int slot = -1;                    // row of the I/O and result tables
    BItem* d_items = nullptr;
    std::vector<long long> units;     // per item: tiles x work units per tile
    std::vector<double> ibytes;       // per item: algorithmic bytes (item_bytes)
    std::vector<int> first[2];        // a new request's first round, by step parity
    std::vector<int> step[2];         // one refinement step, by parity (Jacobi buffer swaps)
    int unpack = -1;
    bool busy = false;
    unsigned long long last_used = 0;
};

struct Req {
    mg_request r;
    uint64_t ticket = 0;
    double t_admit = 0.0;
    int steps = 0;
    bool fresh = true;
    bool cancel = false;          // retire at the start of the next round
    double r0 = 0.0, rel = 1.0;
    Hier* h = nullptr;
};

// Compulsory device-memory bytes of one batched op: every operand it must
// read and every result it must write once (FP32 inner ops 4 B, FP64 outer
// ops 8 B per value), counted over the points of its space.
double item_bytes(const BItem& it) {
    const double pts = (double)it.sp.xr * it.sp.yr * it.sp.zr * it.sp.ncol;
    const double per = it.dim == 3 ? 8.0 : 4.0;   // fine points per coarse point
    const double elems4 = 4.0 * (double)it.n;      // cast / update: n groups of four values
    switch (it.op) {
        case BOP_PACK:
        case BOP_UNPACK: return 16.0 * (double)it.n;
        case BOP_ZERO: return 16.0 * (double)it.n;
        case BOP_REDUCE: return 16.0 * (double)it.n + 32.0;
        case BOP_RES64:
        case BOP_RES64_M: return 24.0 * pts;
        case BOP_CAST: return 12.0 * elems4;
        case BOP_UPDATE: return 20.0 * elems4;
        case BOP_GS:
        case BOP_GS_M:
        case BOP_JAC:
        case BOP_JAC_M:
        case BOP_RES32:
        case BOP_RES32_M: return 12.0 * pts;
        case BOP_GS_ZERO:
        case BOP_JAC_ZERO:
        case BOP_JAC_ZERO_M: return 8.0 * pts;
        case BOP_RESTRICT: return 4.0 * (1.0 + per) * pts;            // sp: coarse points
        case BOP_PROLONG: return 8.0 * pts + 4.0 * pts * 2.0 / (it.sp.ncol * per);   // sp: corrected points
        case BOP_COARSE: return 8.0 * it.m + 8.0 * (double)it.m * it.m;
        default: return 0.0;
    }
}

Key key_of(const mg_request& r) {
    return Key{r.grid.dim, r.grid.n[0], r.opts.smoother, r.opts.nu1, r.opts.nu2, r.opts.post_order, r.opts.omega};
}

mg_opts mixed_opts(const mg_opts& o) {
    mg_opts m = o;
    m.precision = MG_MIXED;
    return m;
}

// Upper bound of the recorded ops: two refinement steps of at most
// 2 (nu1 + nu2) + 4 ops per level plus a handful per step, and the
// load / initial-residual / unpack ops.
size_t items_bound(const mg_grid* g, const mg_opts* o) {
    int L = 1, n = g->n[0];
    while (n > g->coarsest_n) {
        n = (n - 1) / 2 + 1;
        ++L;
    }
    return (size_t)(2 * ((2 * (o->nu1 + o->nu2) + 4) * L + 8) + 8);
}

}  // namespace

struct Server {
    mg_server_opts o{};
    // host executor (mg_server_create_hosted): rounds run through its
    // callbacks, nothing on a device
    bool hosted = false;
    mg_server_executor hx{};
    hipStream_t st = nullptr;
    char* base = nullptr;
    size_t head_bytes = 0;
    Arena arena;
    int max_hier = 0;
    void** d_io = nullptr;            // [slot][2]: f source, u destination
    double* d_results = nullptr;      // [slot][4]: initial (sum, max), latest (sum, max)
    BEntry* d_entries = nullptr;
    size_t entry_cap = 0;
    void** h_io = nullptr;            // pinned mirrors
    double* h_results = nullptr;
    BEntry* h_entries = nullptr;
    std::vector<int> free_slots;
    std::deque<Req> queue;
    uint64_t next_ticket = 0;     // sequence number of the next submitted request
    std::vector<Req> active;
    std::vector<Hier*> hiers;
    std::vector<mg_result> done;
    mg_server_stats stats{};
    unsigned long long tick = 0;
    std::chrono::steady_clock::time_point t0;
    std::string err;
    std::mutex mu;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    int fail(int code, const std::string& m) {
        err = m;
        return code;
    }
    int dev(hipError_t e, const char* what) {
        if (e == hipSuccess) return MG_OK;
        err = std::string(what) + ": " + hipGetErrorString(e);
        return MG_EDEVICE;
    }

    ~Server() {
        for (Hier* h : hiers) {
            delete h->ctx;
            delete h;
        }
        if (h_io) (void)hipHostFree(h_io);
        if (h_results) (void)hipHostFree(h_results);
        if (h_entries) (void)hipHostFree(h_entries);
    }

    static size_t footprint(const mg_grid* g, const mg_opts* o, size_t* ctx_bytes) {
        const mg_opts m = mixed_opts(*o);
        const size_t cb = gran(plan_workspace(g, nullptr, &m, nullptr, false));
        if (ctx_bytes) *ctx_bytes = cb;
        return cb + gran(items_bound(g, o) * sizeof(BItem));
    }

    void release(Hier* h) {
        if (hosted && hx.release) hx.release(hx.user, h->slot);
        arena.release(h->off, h->bytes);
        free_slots.push_back(h->slot);
        delete h->ctx;
        hiers.erase(std::find(hiers.begin(), hiers.end(), h));
        delete h;
        stats.evictions++;
    }

    // Free idle hierarchies, least recently used first, until `bytes` fit.
    bool make_room(size_t bytes, size_t* off) {
        while (!arena.alloc(bytes, off)) {
            Hier* lru = nullptr;
            for (Hier* h : hiers)
                if (!h->busy && (!lru || h->last_used < lru->last_used)) lru = h;
            if (!lru) return false;
            release(lru);
        }
        return true;
    }

    int build(const mg_request& r, Hier** out) {
        *out = nullptr;
        if (free_slots.empty()) {
            Hier* lru = nullptr;
            for (Hier* h : hiers)
                if (!h->busy && (!lru || h->last_used < lru->last_used)) lru = h;
            if (!lru) return MG_ENOMEM;
            release(lru);
        }
        size_t ctx_bytes = 0;
        const size_t fb = footprint(&r.grid, &r.opts, &ctx_bytes);
        size_t off = 0;
        if (!make_room(fb, &off)) return MG_ENOMEM;
        Hier* h = new Hier();
        h->key = key_of(r);
        h->off = off;
        h->bytes = fb;
        h->ctx_bytes = ctx_bytes;
        h->slot = free_slots.back();
        free_slots.pop_back();
        if (hosted) {
            const int rc = hx.build(hx.user, h->slot, &r);
            if (rc) {
                arena.release(off, fb);
                free_slots.push_back(h->slot);
                delete h;
                return fail(rc, "host executor: build");
            }
            hiers.push_back(h);
            stats.hierarchies_built++;
            *out = h;
            return MG_OK;
        }
        const mg_opts m = mixed_opts(r.opts);
        std::string why;
        int rc = setup_ctx(&r.grid, nullptr, &m, base + head_bytes + off, ctx_bytes, st, false, &h->ctx, &why);
        if (rc) {
            arena.release(off, fb);
            free_slots.push_back(h->slot);
            delete h;
            return fail(rc, "hierarchy setup: " + why);
        }
        rc = record_programs(h);
        if (rc) {
            delete h->ctx;
            arena.release(off, fb);
            free_slots.push_back(h->slot);
            delete h;
            return rc;
        }
        hiers.push_back(h);
        stats.hierarchies_built++;
        *out = h;
        return MG_OK;
    }

    int record_programs(Hier* h) {
        Ctx* c = h->ctx;
        std::vector<BItem> items;
        const Level& l0 = c->lv[0];
        const long long nat = (long long)l0.g.n * l0.g.n * (l0.g.dim == 3 ? l0.g.n : 1);
        void* const* io = d_io + 2 * h->slot;
        double* res = d_results + 4 * h->slot;
        // load the right-hand side and zero the iterate
        BItem pk = c->item(BOP_PACK, 0);
        pk.n = nat;
        pk.tiles = (nat + 255) / 256;
        pk.a = l0.f[0];
        pk.io = io;
        items.push_back(pk);
        BItem zr = c->item(BOP_ZERO, 0);
        zr.n = (long long)(l0.field_bytes[0] / 16);
        zr.tiles = (zr.n + 255) / 256;
        zr.a = l0.u[0];
        items.push_back(zr);
        // initial residual and its norm -> res[0..1]
        c->rec = &items;
        c->rec_res = res;
        const size_t init_begin = items.size();
        int rc = c->residual_cast(true);
        const size_t init_end = items.size();
        // refinement steps, norms -> res[2..3]; record two so that Jacobi
        // double buffers return to their starting state after the pair
        c->rec_res = res + 2;
        size_t sb[3];
        for (int p = 0; p < 2 && !rc; ++p) {
            sb[p] = items.size();
            rc = c->refine_step();
            if (!rc) rc = c->residual_cast(false);
        }
        sb[2] = items.size();
        c->rec = nullptr;
        c->rec_res = nullptr;
        if (rc) return fail(rc, "recording: " + c->err);
        BItem up = c->item(BOP_UNPACK, 0);
        up.n = nat;
        up.tiles = (nat + 255) / 256;
        up.a = l0.u[0];
        up.io = io;
        items.push_back(up);
        h->unpack = (int)items.size() - 1;
        for (int p = 0; p < 2; ++p) {
            h->step[p].clear();
            for (size_t i = sb[p]; i < sb[p + 1]; ++i) h->step[p].push_back((int)i);
            h->first[p] = {0, 1};
            for (size_t i = init_begin; i < init_end; ++i) h->first[p].push_back((int)i);
            h->first[p].insert(h->first[p].end(), h->step[p].begin(), h->step[p].end());
        }
        if (items.size() > items_bound(&c->grid, &c->opts) || h->first[0].size() > (size_t)kMaxProgram)
            return fail(MG_EINVAL, "program larger than its bound");
        h->units.clear();
        h->ibytes.clear();
        for (BItem& it : items) {
            if (it.w < 1) it.w = 1;
            h->units.push_back(it.tiles * it.w);
            h->ibytes.push_back(item_bytes(it));
        }
        h->d_items = reinterpret_cast<BItem*>(base + head_bytes + h->off + h->ctx_bytes);
        rc = dev(hipMemcpyAsync(h->d_items, items.data(), items.size() * sizeof(BItem), hipMemcpyHostToDevice, st),
                 "upload program");
        if (!rc) rc = dev(hipStreamSynchronize(st), "sync");
        return rc;
    }

    void admit() {
        while (!queue.empty() && (int)active.size() < o.max_slots) {
            Req& q = queue.front();
            const Key k = key_of(q.r);
            Hier* h = nullptr;
            for (Hier* c : hiers)
                if (!c->busy && c->key == k && (!h || c->last_used > h->last_used)) h = c;
            if (!h) {
                const int rc = build(q.r, &h);
                if (rc == MG_ENOMEM && !active.empty()) break;   // wait for memory to free up
                if (rc) {   // cannot ever be admitted: report it as finished with the error
                    mg_result res{};
                    res.id = q.r.id;
                    res.ticket = q.ticket;
                    res.status = rc;
                    res.t_arrive = q.r.t_arrive;
                    res.t_admit = res.t_done = now();
                    done.push_back(res);
                    queue.pop_front();
                    continue;
                }
            }
            h->busy = true;
            h->last_used = ++tick;
            q.h = h;
            q.t_admit = now();
            if (!hosted) {
                h_io[2 * h->slot] = const_cast<double*>(q.r.f);
                h_io[2 * h->slot + 1] = q.r.u_out;
            }
            active.push_back(q);
            queue.pop_front();
            stats.admitted++;
        }
    }

    int launch_round(const std::vector<const std::vector<int>*>& progs, const std::vector<Hier*>& hs) {
        size_t maxlen = 0;
        for (const auto* p : progs) maxlen = std::max(maxlen, p->size());
        struct L {
            size_t start;
            int count;
            long long total;
        };
        std::vector<L> launches;
        size_t ne = 0;
        for (size_t k = 0; k < maxlen; ++k) {
            L l{ne, 0, 0};
            for (size_t j = 0; j < progs.size(); ++j) {
                if (k >= progs[j]->size()) continue;
                if (ne >= entry_cap) return fail(MG_ENOMEM, "launch table full");
                const int idx = (*progs[j])[k];
                h_entries[ne].item = hs[j]->d_items + idx;
                h_entries[ne].prefix = l.total;
                l.total += hs[j]->units[(size_t)idx];
                stats.algorithmic_bytes += hs[j]->ibytes[(size_t)idx];
                ++l.count;
                ++ne;
            }
            launches.push_back(l);
        }
        int rc = dev(hipMemcpyAsync(d_entries, h_entries, ne * sizeof(BEntry), hipMemcpyHostToDevice, st),
                     "upload launch table");
        for (const L& l : launches) {
            if (rc) break;
            rc = dev(launch_batch(d_entries + l.start, l.count, l.total, st), "batched launch");
            stats.launches++;
        }
        return rc;
    }

    // Retire without further work: the result of a request that never ran
    // or stops here (cancelled, or still queued at its deadline).
    void retire_idle(const Req& q, int status) {
        mg_result res{};
        res.id = q.r.id;
        res.ticket = q.ticket;
        res.status = status;
        res.steps = q.steps;
        res.relres = q.rel;
        res.t_arrive = q.r.t_arrive;
        res.t_admit = q.h ? q.t_admit : 0.0;
        res.t_done = now();
        done.push_back(res);
        if (q.h) {
            q.h->busy = false;
            q.h->last_used = ++tick;
        }
        stats.completed++;
    }

    // Cancellations in flight, and queued requests past their deadline.
    void sweep() {
        std::vector<Req> keep;
        for (Req& q : active) {
            if (q.cancel) retire_idle(q, MG_ECANCELED);
            else keep.push_back(q);
        }
        active.swap(keep);
        const double t = now();
        for (auto it = queue.begin(); it != queue.end();) {
            if (it->r.deadline > 0.0 && t >= it->r.deadline) {
                retire_idle(*it, MG_ETIMEDOUT);
                it = queue.erase(it);
            } else {
                ++it;
            }
        }
    }

    int cancel(uint64_t ticket) {
        for (auto it = queue.begin(); it != queue.end(); ++it)
            if (it->ticket == ticket) {
                retire_idle(*it, MG_ECANCELED);
                queue.erase(it);
                return MG_OK;
            }
        for (Req& q : active)
            if (q.ticket == ticket && !q.cancel) {
                q.cancel = true;
                return MG_OK;
            }
        return MG_EINVAL;
    }

    // One refinement step of every active request on the device: one
    // batched launch per op position, then the norms of every slot.
    int device_round(std::vector<double>& norms) {
        int rc = dev(hipMemcpyAsync(d_io, h_io, (size_t)max_hier * 2 * sizeof(void*), hipMemcpyHostToDevice, st),
                     "upload io");
        if (rc) return rc;
        std::vector<const std::vector<int>*> progs;
        std::vector<Hier*> hs;
        for (Req& q : active) {
            const int par = q.steps & 1;
            progs.push_back(q.fresh ? &q.h->first[par] : &q.h->step[par]);
            hs.push_back(q.h);
        }
        rc = launch_round(progs, hs);
        if (!rc)
            rc = dev(hipMemcpyAsync(h_results, d_results, (size_t)max_hier * 4 * sizeof(double),
                                    hipMemcpyDeviceToHost, st),
                     "read norms");
        if (!rc) rc = dev(hipStreamSynchronize(st), "sync");
        if (rc) return rc;
        for (size_t i = 0; i < active.size(); ++i) {
            const double* rs = h_results + 4 * active[i].h->slot;
            norms[2 * i] = rs[0];
            norms[2 * i + 1] = rs[2];
        }
        return MG_OK;
    }

    // The same step through the host executor.
    int host_round(std::vector<double>& norms) {
        std::vector<int> slots, first;
        std::vector<mg_request> reqs;
        for (const Req& q : active) {
            slots.push_back(q.h->slot);
            first.push_back(q.fresh ? 1 : 0);
            reqs.push_back(q.r);
        }
        const int rc = hx.step(hx.user, (int)active.size(), slots.data(), first.data(), reqs.data(), norms.data());
        return rc ? fail(rc, "host executor: step") : MG_OK;
    }

    int round(int* in_flight, int* queued) {
        sweep();
        admit();
        if (!active.empty()) {
            // norms[2 i], norms[2 i + 1]: sums of squares of active[i]'s
            // initial residual (first step) and of its residual now
            std::vector<double> norms(2 * active.size(), 0.0);
            int rc = hosted ? host_round(norms) : device_round(norms);
            if (rc) return rc;
            stats.rounds++;
            // retire converged requests
            std::vector<Req> keep, fin;
            std::vector<int> status;
            for (size_t i = 0; i < active.size(); ++i) {
                Req& q = active[i];
                if (q.fresh) {
                    q.r0 = std::sqrt(norms[2 * i]);
                    q.fresh = false;
                }
                q.steps++;
                q.rel = q.r0 > 0.0 ? std::sqrt(norms[2 * i + 1]) / q.r0 : 0.0;
                int stt = 1;
                if (!std::isfinite(q.r0) || !std::isfinite(q.rel)) stt = MG_ENONFINITE;
                else if (q.rel <= q.r.tol) stt = MG_OK;
                else if (q.steps >= q.r.opts.max_cycles) stt = MG_ENOTCONV;
                else if (q.r.deadline > 0.0 && now() >= q.r.deadline) stt = MG_ETIMEDOUT;
                if (stt == 1) {
                    keep.push_back(q);
                } else {
                    fin.push_back(q);
                    status.push_back(stt);
                }
            }
            if (hosted) {
                for (size_t i = 0; i < fin.size(); ++i) {
                    rc = hx.finish(hx.user, fin[i].h->slot, &fin[i].r);
                    if (rc) return fail(rc, "host executor: finish");
                }
            } else if (!fin.empty()) {
                std::vector<std::vector<int>> one(fin.size());
                std::vector<const std::vector<int>*> up;
                std::vector<Hier*> uh;
                for (size_t i = 0; i < fin.size(); ++i) {
                    one[i] = {fin[i].h->unpack};
                    up.push_back(&one[i]);
                    uh.push_back(fin[i].h);
                }
                rc = launch_round(up, uh);
                if (!rc) rc = dev(hipStreamSynchronize(st), "sync");
                if (rc) return rc;
            }
            if (!fin.empty()) {
                const double t = now();
                for (size_t i = 0; i < fin.size(); ++i) {
                    mg_result res;
                    res.id = fin[i].r.id;
                    res.ticket = fin[i].ticket;
                    res.status = status[i];
                    res.steps = fin[i].steps;
                    res.relres = fin[i].rel;
                    res.t_arrive = fin[i].r.t_arrive;
                    res.t_admit = fin[i].t_admit;
                    res.t_done = t;
                    done.push_back(res);
                    fin[i].h->busy = false;
                    fin[i].h->last_used = ++tick;
                    stats.completed++;
                }
            }
            active.swap(keep);
        }
        if (in_flight) *in_flight = (int)active.size();
        if (queued) *queued = (int)queue.size();
        return MG_OK;
    }
};

}  // namespace mg

using mg::Server;

extern "C" {

int mg_server_footprint(const mg_grid* g, const mg_opts* o, size_t* bytes) {
    if (!g || !o || !bytes) return MG_EINVAL;
    mg_opts m = *o;
    m.precision = MG_MIXED;
    size_t b = 0;
    int rc = mg_workspace_bytes(g, nullptr, &m, &b);
    if (rc) return rc;
    if (g->centering != MG_NODE) return MG_EINVAL;
    *bytes = Server::footprint(g, o, nullptr);
    return MG_OK;
}

int mg_server_create(const mg_server_opts* o, mg_server** out) {
    if (!o || !out) return MG_EINVAL;
    *out = nullptr;
    if (!o->d_arena || reinterpret_cast<uintptr_t>(o->d_arena) % 256 || o->max_slots < 1 ||
        o->max_slots > 4096 || o->max_queue < 1)
        return MG_EINVAL;
    Server* s = new (std::nothrow) Server();
    if (!s) return MG_ENOMEM;
    s->o = *o;
    s->st = static_cast<hipStream_t>(o->hip_stream);
    s->base = static_cast<char*>(o->d_arena);
    s->max_hier = std::min(4 * o->max_slots, 16384);
    s->entry_cap = (size_t)mg::kMaxProgram * (size_t)o->max_slots;
    const size_t io_b = mg::gran((size_t)s->max_hier * 2 * sizeof(void*));
    const size_t res_b = mg::gran((size_t)s->max_hier * 4 * sizeof(double));
    const size_t ent_b = mg::gran(s->entry_cap * sizeof(mg::BEntry));
    s->head_bytes = io_b + res_b + ent_b;
    if (o->arena_bytes <= s->head_bytes) {
        delete s;
        return MG_ENOMEM;
    }
    s->d_io = reinterpret_cast<void**>(s->base);
    s->d_results = reinterpret_cast<double*>(s->base + io_b);
    s->d_entries = reinterpret_cast<mg::BEntry*>(s->base + io_b + res_b);
    s->arena.init((o->arena_bytes - s->head_bytes) / mg::kGranule * mg::kGranule);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_io), io_b, 0) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_results), res_b, 0) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_entries), ent_b, 0) != hipSuccess) {
        delete s;
        return MG_EDEVICE;
    }
    std::memset(s->h_io, 0, io_b);
    std::memset(s->h_results, 0, res_b);
    for (int i = s->max_hier - 1; i >= 0; --i) s->free_slots.push_back(i);
    if (s->dev(mg::launch_zero(s->base, s->head_bytes, s->st), "zero head") ||
        s->dev(hipStreamSynchronize(s->st), "sync")) {
        delete s;
        return MG_EDEVICE;
    }
    s->t0 = std::chrono::steady_clock::now();
    *out = reinterpret_cast<mg_server*>(s);
    return MG_OK;
}

int mg_server_create_hosted(const mg_server_opts* o, const mg_server_executor* ex, mg_server** out) {
    if (!o || !ex || !out) return MG_EINVAL;
    *out = nullptr;
    if (!ex->build || !ex->step || !ex->finish || o->max_slots < 1 || o->max_slots > 4096 || o->max_queue < 1 ||
        o->arena_bytes < mg::kGranule)
        return MG_EINVAL;
    Server* s = new (std::nothrow) Server();
    if (!s) return MG_ENOMEM;
    s->o = *o;
    s->o.d_arena = nullptr;
    s->o.hip_stream = nullptr;
    s->hosted = true;
    s->hx = *ex;
    s->max_hier = std::min(4 * o->max_slots, 16384);
    s->arena.init(o->arena_bytes / mg::kGranule * mg::kGranule);
    for (int i = s->max_hier - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->t0 = std::chrono::steady_clock::now();
    *out = reinterpret_cast<mg_server*>(s);
    return MG_OK;
}

void mg_server_destroy(mg_server* h) {
    Server* s = reinterpret_cast<Server*>(h);
    if (!s) return;
    if (!s->hosted) (void)hipStreamSynchronize(s->st);
    delete s;
}

double mg_server_clock(const mg_server* h) {
    const Server* s = reinterpret_cast<const Server*>(h);
    return s ? s->now() : 0.0;
}

int mg_server_submit(mg_server* h, const mg_request* r, uint64_t* ticket) {
    Server* s = reinterpret_cast<Server*>(h);
    if (!s || !r) return MG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->grid.centering != MG_NODE || !r->f || !r->u_out || !(r->tol > 0.0))
        return s->fail(MG_EINVAL, "requests need a node grid, device f and u_out, and tol > 0");
    if (r->opts.cycle != MG_CYCLE_V) return s->fail(MG_EINVAL, "the server runs V-cycles");
    size_t ws = 0;
    mg_opts m = r->opts;
    m.precision = MG_MIXED;
    if (mg_workspace_bytes(&r->grid, nullptr, &m, &ws) != MG_OK) return s->fail(MG_EINVAL, "invalid grid or options");
    if (Server::footprint(&r->grid, &r->opts, nullptr) > s->arena.cap)
        return s->fail(MG_ENOMEM, "request larger than the arena");
    if ((int)s->queue.size() >= s->o.max_queue) return s->fail(MG_EBUSY, "queue full");
    mg::Req q;
    q.r = *r;
    q.r.opts.precision = MG_MIXED;
    q.ticket = s->next_ticket++;
    s->queue.push_back(q);
    if (ticket) *ticket = q.ticket;
    return MG_OK;
}

int mg_server_cancel(mg_server* h, uint64_t ticket) {
    Server* s = reinterpret_cast<Server*>(h);
    if (!s) return MG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const int rc = s->cancel(ticket);
    return rc ? s->fail(rc, "no queued or running request with this ticket") : MG_OK;
}

int mg_server_step(mg_server* h, int* in_flight, int* queued) {
    Server* s = reinterpret_cast<Server*>(h);
    if (!s) return MG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    return s->round(in_flight, queued);
}

int mg_server_poll(mg_server* h, mg_result* out, int cap, int* n) {
    Server* s = reinterpret_cast<Server*>(h);
    if (!s || !n || (cap > 0 && !out)) return MG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const int k = std::min(cap, (int)s->done.size());
    for (int i = 0; i < k; ++i) out[i] = s->done[(size_t)i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    return MG_OK;
}

int mg_server_get_stats(const mg_server* h, mg_server_stats* st) {
    const Server* s = reinterpret_cast<const Server*>(h);
    if (!s || !st) return MG_EINVAL;
    *st = s->stats;
    st->arena_peak_bytes = s->arena.peak;
    st->arena_used_bytes = s->arena.used;
    st->in_flight = (int)s->active.size();
    st->queued = (int)s->queue.size();
    st->resident = (int)s->hiers.size();
    return MG_OK;
}

const char* mg_server_last_error(const mg_server* h) {
    const Server* s = reinterpret_cast<const Server*>(h);
    return s ? s->err.c_str() : "null server";
}

}  // extern "C"
