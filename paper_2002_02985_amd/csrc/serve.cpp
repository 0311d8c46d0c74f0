// Request server: continuous batching of energy+potential, force and
// optimisation requests for many cells on one device.  Worker slots (one
// thread and one non-blocking stream each) take requests from a shared queue
// as slots and memory free up, so requests admitted while others run overlap
// with them on the device.  Each cell's grid, and with it its density, stays
// resident between requests for warm starts across MD frames; admission is by
// device-memory footprint (policy in serve_sched.hpp).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_set>
#include <unordered_map>
#include <vector>

#include "../../include/ofdft.h"
#include "internal.hpp"
#include "serve_sched.hpp"

namespace {

using Clock = std::chrono::steady_clock;

ofdft_status fail(ofdft_status st, const std::string &msg)
{
    ofdft_internal::set_error(msg);
    return st;
}

// Deep copy of a cell descriptor (the descriptor points into the vectors).
struct CellCopy {
    ofdft_cell_desc d{};
    std::vector<double> pos, Z, rc;
    std::vector<int32_t> species;

    void assign(const ofdft_cell_desc &c)
    {
        d = c;
        pos.assign(c.pos ? c.pos : nullptr, c.pos ? c.pos + 3 * (size_t)std::max(c.natoms, 0) : nullptr);
        species.assign(c.species ? c.species : nullptr,
                       c.species ? c.species + std::max(c.natoms, 0) : nullptr);
        Z.assign(c.Z ? c.Z : nullptr, c.Z ? c.Z + std::max(c.nspecies, 0) : nullptr);
        rc.assign(c.rc ? c.rc : nullptr, c.rc ? c.rc + std::max(c.nspecies, 0) : nullptr);
        d.pos = pos.data();
        d.species = species.data();
        d.Z = Z.data();
        d.rc = rc.data();
    }
    void assign(const CellCopy &o) { assign(o.d); }
    long long npoints() const { return (long long)d.n[0] * d.n[1] * d.n[2]; }
};

bool same_functional(const ofdft_functional_desc &a, const ofdft_functional_desc &b)
{
    return a.terms == b.terms && a.lambda_vw == b.lambda_vw && a.alpha == b.alpha &&
           a.beta == b.beta && a.kf_wt == b.kf_wt && a.nk == b.nk && a.kf_min == b.kf_min &&
           a.kf_max == b.kf_max && a.knot_spacing == b.knot_spacing && a.nl_mode == b.nl_mode &&
           a.precision == b.precision && a.rho_floor == b.rho_floor &&
           a.nl_kernel == b.nl_kernel;
}

// Everything but the atom positions: a grid built for one serves the other.
bool same_shape(const CellCopy &a, const ofdft_functional_desc &fa, const CellCopy &b,
                const ofdft_functional_desc &fb)
{
    if (std::memcmp(a.d.lattice, b.d.lattice, sizeof(a.d.lattice)) != 0) return false;
    for (int k = 0; k < 3; ++k)
        if (a.d.n[k] != b.d.n[k]) return false;
    return a.d.natoms == b.d.natoms && a.d.nspecies == b.d.nspecies && a.d.nelec == b.d.nelec &&
           a.d.sf_method == b.d.sf_method && a.d.pme_order == b.d.pme_order &&
           a.species == b.species && a.Z == b.Z && a.rc == b.rc && same_functional(fa, fb);
}

enum JobState { QUEUED, RUNNING, DONE };

struct Job {
    uint64_t ticket = 0, cell_id = 0;
    int kind = 0;
    CellCopy cell;
    ofdft_functional_desc func{};
    ofdft_opt_params opt{};
    std::vector<double> rho;
    uint64_t need = 0;
    JobState state = QUEUED;
    std::atomic<int> cancel{0};
    ofdft_status status = OFDFT_PENDING;
    std::string err;
    ofdft_opt_result res{};
    std::vector<double> v, f;
    Clock::time_point t_submit, t_start, t_end;
};

struct Res {
    uint64_t cell_id = 0;
    ofdft_grid *g = nullptr;
    uint64_t bytes = 0;
    bool busy = false;
    // chosen for eviction: its density is being saved and the grid destroyed
    // by a worker outside the lock; it stays busy (requests of its cell wait)
    // and its bytes stay counted until then
    bool evicting = false;
    uint64_t last_use = 0;
    bool has_density = false;
    CellCopy cell;
    ofdft_functional_desc func{};
};

struct SavedDensity {
    int32_t n[3] = {0, 0, 0};
    std::vector<double> rho;
    uint64_t stamp = 0;   // order of saving, for the host-memory cap
};

// host bytes of saved densities kept at most; the least recently saved go
// first beyond it
constexpr uint64_t SAVED_CAP_BYTES = 8ull << 30;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct ofdft_server {
    int device = 0;
    uint64_t budget = 0;
    int max_inflight = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Job>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;   // unreleased tickets
    std::vector<std::unique_ptr<Res>> res;
    uint64_t used = 0, peak = 0, clock = 0, next_ticket = 1;
    // bytes of admitted new grids not yet allocated: their worker first saves
    // and frees the grids it evicts (still counted in used meanwhile), so the
    // device holds at most used - unalloc bytes; the peak records that
    uint64_t unalloc = 0;
    int running = 0;
    bool stop = false;
    uint64_t n_sub = 0, n_done = 0, n_fail = 0, n_cancel = 0;
    std::vector<double> lat_ms, queue_ms;
    std::vector<ofdft_ctx *> ctxs;
    std::vector<std::thread> workers;
    // densities of evicted cells, kept in host memory and handed back as the
    // starting density when the cell's grid is built again (same grid shape)
    std::unordered_map<uint64_t, SavedDensity> saved;
    uint64_t saved_bytes = 0, saved_clock = 0;
    // continuous batching of energy+potential requests across cells
    int batch_max = 8;       // energy+potential requests per batch
    int opt_batch_max = 1;   // optimisation requests per lockstep batch (off: measured
                             // slower than running them on separate worker slots)
    uint64_t n_batches = 0, n_batched = 0;
};

namespace {

// The resident grid of a cell, not counting one that is being evicted
int find_resident(const ofdft_server *s, uint64_t cell_id)
{
    for (size_t r = 0; r < s->res.size(); ++r)
        if (s->res[r]->cell_id == cell_id && !s->res[r]->evicting) return (int)r;
    return -1;
}

// For the admission views: the cell's resident grid, else the grid of it that
// is being evicted (busy, so that the cell's requests wait until its density
// has been saved), else -1
int find_resident_or_evicting(const ofdft_server *s, uint64_t cell_id)
{
    const int r = find_resident(s, cell_id);
    if (r >= 0) return r;
    for (size_t k = 0; k < s->res.size(); ++k)
        if (s->res[k]->cell_id == cell_id) return (int)k;
    return -1;
}

// Keeps an evicted cell's density (under the lock), dropping the least
// recently saved ones beyond the host-memory cap
void save_density(ofdft_server *s, uint64_t cell_id, SavedDensity &&h)
{
    auto old = s->saved.find(cell_id);
    if (old != s->saved.end()) {
        s->saved_bytes -= old->second.rho.size() * sizeof(double);
        s->saved.erase(old);
    }
    const uint64_t bytes = h.rho.size() * sizeof(double);
    if (bytes > SAVED_CAP_BYTES) return;
    while (s->saved_bytes + bytes > SAVED_CAP_BYTES && !s->saved.empty()) {
        auto lru = s->saved.begin();
        for (auto it = s->saved.begin(); it != s->saved.end(); ++it)
            if (it->second.stamp < lru->second.stamp) lru = it;
        s->saved_bytes -= lru->second.rho.size() * sizeof(double);
        s->saved.erase(lru);
    }
    h.stamp = ++s->saved_clock;
    s->saved_bytes += bytes;
    s->saved[cell_id] = std::move(h);
}

// Runs one request on resident grid r (created here if it has none) on the
// worker's context.  Called without the server lock; r is owned by this
// worker while busy.  saved: the density kept for this cell when its grid
// was evicted (empty if none), the start of a request that brings none.
// rho0 = N_e / V at every point of the request's grid
std::vector<double> uniform_density(const Job &job)
{
    const double(&a)[3][3] = job.cell.d.lattice;
    const double V = std::fabs(a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                               a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                               a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]));
    return std::vector<double>((size_t)job.cell.npoints(), job.cell.d.nelec / V);
}

// A resident grid brought to a batched request on this worker's context:
// the atoms moved in place, the density given with the request, else the
// resident one (a cold optimisation, or a grid without one: the uniform one)
ofdft_status prepare_resident(Job &job, Res &r, ofdft_ctx *ctx)
{
    ofdft_internal::bind_context(r.g, ctx);
    ofdft_status st = OFDFT_OK;
    if (r.cell.pos != job.cell.pos) {
        st = ofdft_internal::set_positions(r.g, job.cell.pos.data());
        if (st == OFDFT_OK) r.cell.assign(job.cell);
    }
    const bool cold_opt = job.kind == OFDFT_REQ_OPTIMIZE && !job.opt.warm;
    if (st == OFDFT_OK) {
        if (!job.rho.empty()) {
            st = ofdft_set_density(r.g, job.rho.data());
        } else if (!r.has_density || cold_opt) {
            const std::vector<double> u = uniform_density(job);
            st = ofdft_set_density(r.g, u.data());
        }
    }
    if (st == OFDFT_OK) r.has_density = true;
    return st;
}

void execute(Job &job, Res &r, ofdft_ctx *ctx, const SavedDensity &saved)
{
    ofdft_status st = OFDFT_OK;
    bool fresh = false;
    if (!r.g) {
        st = ofdft_grid_create(ctx, &job.cell.d, &job.func, &r.g);
        if (st == OFDFT_OK) {
            r.cell.assign(job.cell);
            r.func = job.func;
            r.has_density = false;
            fresh = true;
            // the worker streams can be captured: evaluations replay graphs
            (void)ofdft_grid_set_graphs(r.g, 1);
        }
    } else {
        ofdft_internal::bind_context(r.g, ctx);
        if (r.cell.pos != job.cell.pos) {
            st = ofdft_internal::set_positions(r.g, job.cell.pos.data());
            if (st == OFDFT_OK) r.cell.assign(job.cell);
        }
    }
    ofdft_grid *g = r.g;
    const bool cold_opt = job.kind == OFDFT_REQ_OPTIMIZE && !job.opt.warm;
    if (st == OFDFT_OK) {
        ofdft_internal::set_cancel(g, &job.cancel);
        if (!job.rho.empty()) {
            st = ofdft_set_density(g, job.rho.data());
        } else if (!r.has_density && !cold_opt && !saved.rho.empty() &&
                   saved.n[0] == job.cell.d.n[0] && saved.n[1] == job.cell.d.n[1] &&
                   saved.n[2] == job.cell.d.n[2]) {
            st = ofdft_set_density(g, saved.rho.data());
        } else if (!r.has_density || cold_opt) {
            const std::vector<double> u = uniform_density(job);
            st = ofdft_set_density(g, u.data());
        }
        if (st == OFDFT_OK) r.has_density = true;
        // a shape seen for the first time: tune its launch schedule once
        if (st == OFDFT_OK && fresh && !ofdft_internal::has_tuning(g))
            st = ofdft_grid_tune(g, nullptr);
    }
    if (st == OFDFT_OK) {
        job.res.evals = 1;
        switch (job.kind) {
        case OFDFT_REQ_EP:
            job.v.resize((size_t)job.cell.npoints());
            st = ofdft_energy_potential(g, nullptr, job.v.data(), &job.res.e);
            break;
        case OFDFT_REQ_FORCES:
            st = ofdft_energy_potential(g, nullptr, nullptr, &job.res.e);
            if (st == OFDFT_OK) {
                job.f.resize(3 * (size_t)job.cell.d.natoms);
                st = ofdft_forces(g, job.f.data());
            }
            break;
        default:
            st = ofdft_optimize(g, &job.opt, &job.res);
            break;
        }
    }
    if (g) ofdft_internal::set_cancel(g, nullptr);
    if (st != OFDFT_OK) job.err = ofdft_last_error();
    if (job.cancel.load()) {
        st = OFDFT_ECANCELLED;
        job.err = "request cancelled";
        job.v.clear();
        job.f.clear();
    }
    job.status = st;
}

// Runs energy+potential requests of several resident cells (one grid shape
// and functional) as one batched evaluation led by the first one's grid.
// Called without the server lock; every grid is owned by this worker while
// busy.  Falls back to one request at a time if the batch cannot run.
void execute_batch(const std::vector<Job *> &jobs, const std::vector<Res *> &res, ofdft_ctx *ctx)
{
    const size_t n = jobs.size();
    std::vector<ofdft_grid *> grids(n);
    std::vector<double *> vptr(n);
    std::vector<ofdft_energy> e(n);
    ofdft_status st = OFDFT_OK;
    for (size_t b = 0; b < n && st == OFDFT_OK; ++b) {
        Job &job = *jobs[b];
        Res &r = *res[b];
        st = prepare_resident(job, r, ctx);
        grids[b] = r.g;
        job.v.resize((size_t)job.cell.npoints());
        vptr[b] = job.v.data();
    }
    if (st == OFDFT_OK) st = ofdft_energy_potential_multi(grids.data(), (int32_t)n, vptr.data(), e.data());
    if (st != OFDFT_OK) {   // one at a time (each request gets its own status)
        for (size_t b = 0; b < n; ++b) {
            Job &job = *jobs[b];
            job.status = ofdft_energy_potential(res[b]->g, nullptr, job.v.data(), &job.res.e);
            job.res.evals = 1;
            if (job.status != OFDFT_OK) job.err = ofdft_last_error();
        }
    } else {
        for (size_t b = 0; b < n; ++b) {
            jobs[b]->res.e = e[b];
            jobs[b]->res.evals = 1;
            jobs[b]->status = OFDFT_OK;
        }
    }
    for (Job *job : jobs)
        if (job->cancel.load()) {
            job->status = OFDFT_ECANCELLED;
            job->err = "request cancelled";
            job->v.clear();
        }
}

// Runs optimisation requests of several resident cells (one grid shape and
// functional) as one lockstep optimisation (their evaluations batched).
// Called without the server lock; every grid is owned by this worker while
// busy.  Falls back to one request at a time if the batch cannot run.
void execute_opt_batch(const std::vector<Job *> &jobs, const std::vector<Res *> &res,
                       ofdft_ctx *ctx)
{
    std::vector<ofdft_grid *> grids;
    std::vector<ofdft_opt_params> prm;
    std::vector<size_t> idx;
    for (size_t b = 0; b < jobs.size(); ++b) {
        Job &job = *jobs[b];
        job.status = prepare_resident(job, *res[b], ctx);
        if (job.status != OFDFT_OK) {
            job.err = ofdft_last_error();
            continue;
        }
        ofdft_internal::set_cancel(res[b]->g, &job.cancel);
        grids.push_back(res[b]->g);
        prm.push_back(job.opt);
        idx.push_back(b);
    }
    const size_t n = grids.size();
    std::vector<ofdft_opt_result> out(n);
    std::vector<ofdft_status> sts(n, OFDFT_OK);
    ofdft_status st = OFDFT_EINVAL;
    if (n > 0)
        st = ofdft_optimize_multi(grids.data(), (int32_t)n, prm.data(), out.data(), sts.data());
    const std::string err = ofdft_last_error();
    for (size_t k = 0; k < n; ++k) {
        Job &job = *jobs[idx[k]];
        if (st == OFDFT_OK) {
            job.res = out[k];
            job.status = sts[k];
            if (job.status != OFDFT_OK)
                job.err = job.status == OFDFT_ENOCONV ? "optimisation did not reach the tolerance"
                                                      : err;
        } else {   // one at a time (each request gets its own status)
            job.status = ofdft_optimize(grids[k], &job.opt, &job.res);
            if (job.status != OFDFT_OK) job.err = ofdft_last_error();
        }
        ofdft_internal::set_cancel(grids[k], nullptr);
    }
    for (Job *job : jobs)
        if (job->cancel.load()) {
            job->status = OFDFT_ECANCELLED;
            job->err = "request cancelled";
        }
}

void worker_loop(ofdft_server *s, int w)
{
    ofdft_ctx *ctx = s->ctxs[w];
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->stop && s->queue.empty()) break;
        // views for the admission policy
        std::vector<ofdft_sched::Queued> qv(s->queue.size());
        std::vector<ofdft_sched::Resident> rv(s->res.size());
        for (size_t r = 0; r < s->res.size(); ++r) {
            rv[r].cell_id = s->res[r]->cell_id;
            rv[r].bytes = s->res[r]->bytes;
            rv[r].busy = s->res[r]->busy;
            rv[r].last_use = s->res[r]->last_use;
        }
        for (size_t r = 0; r < s->res.size(); ++r) rv[r].busy |= s->res[r]->evicting;
        for (size_t i = 0; i < s->queue.size(); ++i) {
            const Job &j = *s->queue[i];
            qv[i].cell_id = j.cell_id;
            qv[i].need = j.need;
            qv[i].resident = find_resident_or_evicting(s, j.cell_id);
            if (qv[i].resident >= 0) {
                const Res &r = *s->res[qv[i].resident];
                rv[qv[i].resident].pending = true;
                qv[i].reuse = r.g && !r.evicting && same_shape(r.cell, r.func, j.cell, j.func);
            }
        }
        ofdft_sched::Decision d =
            ofdft_sched::pick(qv, rv, s->used, s->budget, s->running, s->max_inflight);
        if (d.job < 0) {
            s->cv_work.wait(lk);
            continue;
        }
        std::shared_ptr<Job> job = s->queue[d.job];
        // continuous batching: an energy+potential (or optimisation) request
        // on a resident grid takes further queued requests of the same kind
        // of other resident cells with the same grid shape and functional
        // along (each the earliest queued request of its cell, its grid
        // idle), as long as the leader's larger workspace fits in the
        // budget: one batched evaluation, or one lockstep optimisation whose
        // evaluations are batched
        std::vector<std::shared_ptr<Job>> batch;
        std::vector<Res *> batch_res;
        const int bmax = job->kind == OFDFT_REQ_EP ? s->batch_max
                         : job->kind == OFDFT_REQ_OPTIMIZE ? s->opt_batch_max : 1;
        if (bmax > 1 && d.evict.empty()) {
            const int lr = find_resident(s, job->cell_id);
            if (lr >= 0 && s->res[lr]->g && !s->res[lr]->busy &&
                same_shape(s->res[lr]->cell, s->res[lr]->func, job->cell, job->func)) {
                const Res &L = *s->res[lr];
                std::unordered_set<uint64_t> seen;
                seen.insert(job->cell_id);
                for (size_t i = 0; i < s->queue.size() && (int)batch.size() + 1 < bmax; ++i) {
                    if ((int)i == d.job) continue;
                    const Job &j = *s->queue[i];
                    if (!seen.insert(j.cell_id).second) continue;   // not its cell's earliest
                    if (j.kind != job->kind) continue;
                    const int r = find_resident(s, j.cell_id);
                    if (r < 0) continue;
                    Res &R = *s->res[r];
                    if (R.busy || R.evicting || !R.g) continue;
                    if (!same_shape(R.cell, R.func, j.cell, j.func)) continue;
                    if (j.kind == OFDFT_REQ_EP && j.rho.empty() && !R.has_density) continue;
                    if (!same_functional(R.func, L.func) || R.cell.d.n[0] != L.cell.d.n[0] ||
                        R.cell.d.n[1] != L.cell.d.n[1] || R.cell.d.n[2] != L.cell.d.n[2])
                        continue;
                    // the leader's allocations grow to the batch (and stay)
                    if (s->used + ofdft_internal::multi_growth_bytes(L.g, (int)batch.size() + 2) >
                        s->budget)
                        break;
                    batch.push_back(s->queue[i]);
                    batch_res.push_back(&R);
                }
                if (!batch.empty()) {
                    // count the growth now, so that admissions and other
                    // batches made while this one runs see it
                    const uint64_t grow =
                        ofdft_internal::multi_growth_bytes(L.g, (int)batch.size() + 1);
                    s->used += grow;
                    s->res[lr]->bytes += grow;
                    s->peak = std::max(s->peak, s->used - s->unalloc);
                }
            }
        }
        s->queue.erase(s->queue.begin() + d.job);
        for (const auto &bj : batch)
            for (size_t i = 0; i < s->queue.size(); ++i)
                if (s->queue[i] == bj) {
                    s->queue.erase(s->queue.begin() + i);
                    break;
                }
        for (size_t k = 0; k < batch.size(); ++k) {
            batch_res[k]->busy = true;
            batch[k]->state = RUNNING;
            batch[k]->t_start = Clock::now();
        }
        // mark the evicted grids: they stay resident, busy and counted until
        // this worker has saved their densities and destroyed them below
        struct Evicted {
            Res *res;
            ofdft_grid *g;
            uint64_t cell_id;
            bool keep;          // has a density worth restoring
            int32_t n[3];
        };
        std::vector<Evicted> to_free;
        for (int r : d.evict) {
            Res &x = *s->res[r];
            x.evicting = true;
            x.busy = true;
            to_free.push_back({&x, x.g, x.cell_id, x.g && x.has_density,
                               {x.cell.d.n[0], x.cell.d.n[1], x.cell.d.n[2]}});
        }
        Res *r = nullptr;
        uint64_t new_bytes = 0;   // a new grid admitted for this request
        SavedDensity saved;
        const int ri = find_resident(s, job->cell_id);
        if (ri >= 0) {
            r = s->res[ri].get();
        } else {
            auto it = s->saved.find(job->cell_id);
            if (it != s->saved.end()) {
                s->saved_bytes -= it->second.rho.size() * sizeof(double);
                saved = std::move(it->second);
                s->saved.erase(it);
            }
            std::unique_ptr<Res> nr(new Res);
            nr->cell_id = job->cell_id;
            nr->bytes = job->need;
            r = nr.get();
            s->res.push_back(std::move(nr));
            s->used += job->need;
            s->unalloc += job->need;
            new_bytes = job->need;
        }
        r->busy = true;
        s->running++;
        job->state = RUNNING;
        job->t_start = Clock::now();
        lk.unlock();

        // save and free the evicted grids before this request allocates its
        // own, then retire them from the resident set and the byte count
        std::vector<SavedDensity> kept(to_free.size());
        std::vector<bool> ok(to_free.size(), false);
        for (size_t k = 0; k < to_free.size(); ++k) {
            const Evicted &e = to_free[k];
            if (!e.g) continue;
            ofdft_internal::bind_context(e.g, ctx);   // idle: nothing of it is in flight
            if (e.keep) {
                SavedDensity &h = kept[k];
                std::memcpy(h.n, e.n, sizeof(h.n));
                h.rho.resize((size_t)e.n[0] * e.n[1] * e.n[2]);
                ok[k] = ofdft_get_density(e.g, h.rho.data()) == OFDFT_OK;
            }
            ofdft_grid_destroy(e.g);
        }
        if (!to_free.empty()) {
            std::lock_guard<std::mutex> g2(s->mu);
            for (size_t k = 0; k < to_free.size(); ++k) {
                const Evicted &e = to_free[k];
                if (ok[k]) save_density(s, e.cell_id, std::move(kept[k]));
                for (size_t x = 0; x < s->res.size(); ++x)
                    if (s->res[x].get() == e.res) {
                        s->used -= s->res[x]->bytes;
                        s->res.erase(s->res.begin() + x);
                        break;
                    }
            }
            s->cv_work.notify_all();
        }
        {
            std::lock_guard<std::mutex> g2(s->mu);
            s->unalloc -= new_bytes;   // the evictions are done: the new grid may now allocate
            s->peak = std::max(s->peak, s->used - s->unalloc);
        }
        if (batch.empty()) {
            execute(*job, *r, ctx, saved);
        } else {
            std::vector<Job *> jobs{job.get()};
            std::vector<Res *> rs{r};
            for (size_t k = 0; k < batch.size(); ++k) {
                jobs.push_back(batch[k].get());
                rs.push_back(batch_res[k]);
            }
            if (job->kind == OFDFT_REQ_EP) execute_batch(jobs, rs, ctx);
            else execute_opt_batch(jobs, rs, ctx);
        }

        lk.lock();
        if (!batch.empty()) {
            // the leader's growth was counted when the batch was formed; the
            // device's own count can only confirm it
            const uint64_t now = ofdft_grid_device_bytes(r->g);
            if (now > r->bytes) {
                s->used += now - r->bytes;
                r->bytes = now;
            }
            s->peak = std::max(s->peak, s->used - s->unalloc);
            s->n_batched += batch.size() + 1;
            s->n_batches++;
        }
        for (size_t k = 0; k < batch.size(); ++k) {
            Job &bj = *batch[k];
            bj.t_end = Clock::now();
            batch_res[k]->busy = false;
            batch_res[k]->last_use = ++s->clock;
            bj.state = DONE;
            if (bj.status == OFDFT_OK || bj.status == OFDFT_ENOCONV) {
                s->n_done++;
                s->lat_ms.push_back(ms_between(bj.t_submit, bj.t_end));
                s->queue_ms.push_back(ms_between(bj.t_submit, bj.t_start));
            } else if (bj.status == OFDFT_ECANCELLED) {
                s->n_cancel++;
            } else {
                s->n_fail++;
            }
        }
        job->t_end = Clock::now();
        r->busy = false;
        r->last_use = ++s->clock;
        if (!r->g) {   // the grid could not be built: give its memory back
            const int k = find_resident(s, r->cell_id);
            s->used -= r->bytes;
            s->res.erase(s->res.begin() + k);
        }
        s->running--;
        job->state = DONE;
        if (job->status == OFDFT_OK || job->status == OFDFT_ENOCONV) {
            s->n_done++;
            s->lat_ms.push_back(ms_between(job->t_submit, job->t_end));
            s->queue_ms.push_back(ms_between(job->t_submit, job->t_start));
        } else if (job->status == OFDFT_ECANCELLED) {
            s->n_cancel++;
        } else {
            s->n_fail++;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

ofdft_status check_request(const ofdft_request *q)
{
    if (!q) return fail(OFDFT_EINVAL, "null request");
    if (q->kind < OFDFT_REQ_EP || q->kind > OFDFT_REQ_OPTIMIZE)
        return fail(OFDFT_EINVAL, "bad request kind");
    ofdft_status st = ofdft_validate(q->cell, q->func);
    if (st != OFDFT_OK) return st;
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite((&q->cell->lattice[0][0])[k])) return fail(OFDFT_EINVAL, "non-finite lattice");
    for (int s = 0; s < q->cell->nspecies; ++s)
        if (!std::isfinite(q->cell->Z[s]) || !std::isfinite(q->cell->rc[s]))
            return fail(OFDFT_EINVAL, "non-finite species parameters");
    if (q->kind == OFDFT_REQ_OPTIMIZE) {
        if (!q->opt) return fail(OFDFT_EINVAL, "optimisation request without parameters");
        if (!(q->opt->tol > 0) || q->opt->max_iter < 0) return fail(OFDFT_EINVAL, "bad parameters");
    }
    if (q->rho_or_null) {
        const long long N = (long long)q->cell->n[0] * q->cell->n[1] * q->cell->n[2];
        for (long long i = 0; i < N; ++i)
            if (!std::isfinite(q->rho_or_null[i]) || q->rho_or_null[i] < 0)
                return fail(OFDFT_EINVAL, "density has non-finite or negative values");
    }
    return OFDFT_OK;
}

}  // namespace

extern "C" {

ofdft_status ofdft_server_create(ofdft_ctx *ctx, uint64_t hbm_budget_bytes, int32_t max_inflight,
                                 ofdft_server **out)
{
    if (!ctx || !out) return fail(OFDFT_EINVAL, "null argument");
    *out = nullptr;
    if (max_inflight < 1 || max_inflight > 64) return fail(OFDFT_EINVAL, "max_inflight out of range");
    const int dev = ofdft_internal::ctx_device(ctx);
    if (hipSetDevice(dev) != hipSuccess) return fail(OFDFT_EDEVICE, "hipSetDevice failed");
    if (hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(OFDFT_EDEVICE, "hipMemGetInfo failed");
        hbm_budget_bytes = (uint64_t)(0.9 * (double)fr);
    }
    ofdft_server *s = new (std::nothrow) ofdft_server;
    if (!s) return fail(OFDFT_ENOMEM, "host allocation failed");
    s->device = dev;
    s->budget = hbm_budget_bytes;
    s->max_inflight = max_inflight;
    for (int w = 0; w < max_inflight; ++w) {
        ofdft_ctx *c = nullptr;
        ofdft_status st = ofdft_ctx_create(dev, &c);
        if (st != OFDFT_OK) {
            for (ofdft_ctx *x : s->ctxs) ofdft_ctx_destroy(x);
            delete s;
            return st;
        }
        s->ctxs.push_back(c);
    }
    for (int w = 0; w < max_inflight; ++w) s->workers.emplace_back(worker_loop, s, w);
    *out = s;
    return OFDFT_OK;
}

ofdft_status ofdft_serve_submit(ofdft_server *s, const ofdft_request *req, uint64_t *ticket)
{
    if (!s || !ticket) return fail(OFDFT_EINVAL, "null argument");
    *ticket = 0;
    ofdft_status st = check_request(req);
    if (st != OFDFT_OK) return st;
    uint64_t need = 0;
    st = ofdft_footprint_bytes(req->cell, req->func, OFDFT_REQ_OPTIMIZE, &need);
    if (st != OFDFT_OK) return st;
    need += 3 * (uint64_t)req->cell->natoms * sizeof(double);   // forces buffer
    if (need > s->budget)
        return fail(OFDFT_ENOMEM, "request footprint " + std::to_string(need) +
                                      " B exceeds the server budget " + std::to_string(s->budget) + " B");
    auto job = std::make_shared<Job>();
    job->cell_id = req->cell_id;
    job->kind = req->kind;
    job->cell.assign(*req->cell);
    job->func = *req->func;
    if (req->opt) job->opt = *req->opt;
    if (req->rho_or_null) job->rho.assign(req->rho_or_null, req->rho_or_null + job->cell.npoints());
    job->need = need;
    job->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(OFDFT_ECANCELLED, "server is shutting down");
        job->ticket = s->next_ticket++;
        s->jobs[job->ticket] = job;
        s->queue.push_back(job);
        s->n_sub++;
    }
    s->cv_work.notify_one();
    *ticket = job->ticket;
    return OFDFT_OK;
}

ofdft_status ofdft_serve_poll(ofdft_server *s, uint64_t ticket, ofdft_opt_result *res,
                              double *v_or_null, double *f_or_null)
{
    if (!s) return fail(OFDFT_EINVAL, "null argument");
    std::shared_ptr<Job> job;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) return fail(OFDFT_ENOTFOUND, "unknown ticket");
        if (it->second->state != DONE) return OFDFT_PENDING;
        job = it->second;
        s->jobs.erase(it);
    }
    if (res) *res = job->res;
    if (v_or_null && !job->v.empty()) std::memcpy(v_or_null, job->v.data(), job->v.size() * 8);
    if (f_or_null && !job->f.empty()) std::memcpy(f_or_null, job->f.data(), job->f.size() * 8);
    if (job->status != OFDFT_OK) ofdft_internal::set_error(job->err);
    return job->status;
}

ofdft_status ofdft_serve_wait(ofdft_server *s, uint64_t ticket, int32_t timeout_ms)
{
    if (!s) return fail(OFDFT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto done = [&] {
        auto it = s->jobs.find(ticket);
        return it == s->jobs.end() || it->second->state == DONE;
    };
    if (s->jobs.find(ticket) == s->jobs.end()) return fail(OFDFT_ENOTFOUND, "unknown ticket");
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
        return OFDFT_PENDING;
    }
    return OFDFT_OK;
}

ofdft_status ofdft_serve_cancel(ofdft_server *s, uint64_t ticket)
{
    if (!s) return fail(OFDFT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return fail(OFDFT_ENOTFOUND, "unknown ticket");
    Job &j = *it->second;
    j.cancel.store(1);
    if (j.state == QUEUED) {
        for (size_t i = 0; i < s->queue.size(); ++i)
            if (s->queue[i].get() == &j) {
                s->queue.erase(s->queue.begin() + i);
                break;
            }
        j.state = DONE;
        j.status = OFDFT_ECANCELLED;
        j.err = "request cancelled";
        j.t_end = Clock::now();
        s->n_cancel++;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    } else if (j.state == DONE && j.status != OFDFT_ECANCELLED) {
        if (j.status == OFDFT_OK || j.status == OFDFT_ENOCONV) {
            s->n_done--;
        } else {
            s->n_fail--;
        }
        s->n_cancel++;
        j.status = OFDFT_ECANCELLED;
        j.err = "request cancelled";
        j.v.clear();
        j.f.clear();
    }
    return OFDFT_OK;
}

ofdft_status ofdft_serve_set_batching(ofdft_server *s, int32_t max_ep, int32_t max_opt)
{
    if (!s) return fail(OFDFT_EINVAL, "null server");
    if (max_ep < 1 || max_ep > OFDFT_MULTI_MAX || max_opt < 1 || max_opt > OFDFT_MULTI_MAX)
        return fail(OFDFT_EINVAL, "batch size outside 1..OFDFT_MULTI_MAX");
    std::lock_guard<std::mutex> lk(s->mu);
    s->batch_max = max_ep;
    s->opt_batch_max = max_opt;
    return OFDFT_OK;
}

ofdft_status ofdft_serve_stats_get(ofdft_server *s, ofdft_serve_stats *out)
{
    if (!s || !out) return fail(OFDFT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->n_sub;
    out->completed = s->n_done;
    out->failed = s->n_fail;
    out->cancelled = s->n_cancel;
    out->queued = (int32_t)s->queue.size();
    out->running = s->running;
    out->resident_cells = (int32_t)s->res.size();
    out->max_inflight = s->max_inflight;
    out->resident_bytes = s->used;
    out->peak_bytes = s->peak;
    out->budget_bytes = s->budget;
    out->p50_ms = ofdft_sched::percentile(s->lat_ms, 50.0);
    out->p99_ms = ofdft_sched::percentile(s->lat_ms, 99.0);
    double q = 0;
    for (double x : s->queue_ms) q += x;
    out->mean_queue_ms = s->queue_ms.empty() ? 0.0 : q / (double)s->queue_ms.size();
    out->batches = s->n_batches;
    out->batched_requests = s->n_batched;
    return OFDFT_OK;
}

void ofdft_server_destroy(ofdft_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto &j : s->queue) {
            j->cancel.store(1);
            j->state = DONE;
            j->status = OFDFT_ECANCELLED;
            s->n_cancel++;
        }
        s->queue.clear();
        for (auto &kv : s->jobs) kv.second->cancel.store(1);
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto &r : s->res)
        if (r->g) {
            ofdft_internal::bind_context(r->g, s->ctxs[0]);
            ofdft_grid_destroy(r->g);
        }
    s->res.clear();
    for (ofdft_ctx *c : s->ctxs) ofdft_ctx_destroy(c);
    delete s;
}

}  // extern "C"
