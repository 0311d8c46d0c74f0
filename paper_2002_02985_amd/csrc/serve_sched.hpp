// Admission policy of the request server: which queued request runs next and
// which idle resident grids make room for it.  Plain host C++ with no device
// calls, so that the policy can be exercised on its own.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <unordered_set>
#include <vector>

namespace ofdft_sched {

// A queued request, in submission order.
struct Queued {
    uint64_t cell_id = 0;
    uint64_t need = 0;    // bytes of a new grid for it
    int resident = -1;    // index of its cell's resident grid, -1 if none
    bool reuse = false;   // that resident grid fits the request (same cell shape)
};

// A resident grid.
struct Resident {
    uint64_t cell_id = 0;
    uint64_t bytes = 0;
    bool busy = false;       // a request of this cell is running
    bool pending = false;    // a queued request names this cell
    uint64_t last_use = 0;   // larger is more recent
};

struct Decision {
    int job = -1;               // index into the queue, -1: nothing can start
    std::vector<int> evict;     // resident grids to free before it starts
};

// Picks the next request.  Rules:
//  * no more than max_inflight requests run at once;
//  * requests of one cell run one at a time, in submission order;
//  * a request whose cell has a reusable resident grid needs no memory;
//  * any other request needs `need` bytes: free budget first, then idle
//    resident grids are evicted (its own cell's unusable grid first, then
//    those with nothing queued, least recently used first, then the rest in
//    the same order);
//  * the first request that cannot get its memory holds every later request
//    that needs new memory (no overtaking by smaller requests), while later
//    requests on reusable resident grids still start.
inline Decision pick(const std::vector<Queued> &queue, const std::vector<Resident> &res,
                     uint64_t used, uint64_t budget, int running, int max_inflight)
{
    Decision d;
    if (running >= max_inflight) return d;
    std::unordered_set<uint64_t> seen;
    bool mem_blocked = false;
    for (size_t i = 0; i < queue.size(); ++i) {
        const Queued &q = queue[i];
        if (!seen.insert(q.cell_id).second) continue;   // an earlier request of this cell waits
        if (q.resident >= 0 && res[q.resident].busy) continue;
        if (q.resident >= 0 && q.reuse) {
            d.job = (int)i;
            return d;
        }
        if (mem_blocked) continue;
        std::vector<int> evict;
        uint64_t avail = budget > used ? budget - used : 0;
        if (q.resident >= 0) {
            evict.push_back(q.resident);
            avail += res[q.resident].bytes;
        }
        if (q.need <= avail) {
            d.job = (int)i;
            d.evict = evict;
            return d;
        }
        std::vector<int> idle;
        for (int r = 0; r < (int)res.size(); ++r)
            if (r != q.resident && !res[r].busy) idle.push_back(r);
        std::stable_sort(idle.begin(), idle.end(), [&](int a, int b) {
            if (res[a].pending != res[b].pending) return !res[a].pending;
            return res[a].last_use < res[b].last_use;
        });
        for (int r : idle) {
            evict.push_back(r);
            avail += res[r].bytes;
            if (q.need <= avail) {
                d.job = (int)i;
                d.evict = evict;
                return d;
            }
        }
        mem_blocked = true;
    }
    return d;
}

// Nearest-rank percentile of a sample (p in [0, 100]); 0 for an empty one.
inline double percentile(std::vector<double> v, double p)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t k = (size_t)std::ceil(p / 100.0 * (double)v.size());
    if (k < 1) k = 1;
    if (k > v.size()) k = v.size();
    return v[k - 1];
}

}  // namespace ofdft_sched
