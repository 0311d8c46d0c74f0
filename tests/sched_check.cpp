// Scenario checks of the request server's admission policy (host only).
// Built and run by test_serve_sched.py; prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>

#include "../paper_2002_02985_amd/csrc/serve_sched.hpp"

using namespace ofdft_sched;

static int failures = 0;
#define CHECK(c)                                                                      \
    do {                                                                              \
        if (!(c)) {                                                                   \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);                          \
            ++failures;                                                               \
        }                                                                             \
    } while (0)

static Queued q(uint64_t cell, uint64_t need, int resident = -1, bool reuse = false)
{
    Queued x;
    x.cell_id = cell;
    x.need = need;
    x.resident = resident;
    x.reuse = reuse;
    return x;
}

static Resident r(uint64_t cell, uint64_t bytes, bool busy, bool pending, uint64_t last)
{
    Resident x;
    x.cell_id = cell;
    x.bytes = bytes;
    x.busy = busy;
    x.pending = pending;
    x.last_use = last;
    return x;
}

int main()
{
    {   // arrival order when everything fits
        Decision d = pick({q(1, 10), q(2, 10)}, {}, 0, 100, 0, 4);
        CHECK(d.job == 0 && d.evict.empty());
    }
    {   // all slots taken
        Decision d = pick({q(1, 10)}, {}, 0, 100, 4, 4);
        CHECK(d.job == -1);
    }
    {   // a resident, reusable grid needs no memory even with the budget used up
        Decision d = pick({q(7, 60, 0, true)}, {r(7, 60, false, true, 1)}, 100, 100, 0, 4);
        CHECK(d.job == 0 && d.evict.empty());
    }
    {   // one request per cell at a time: the cell is busy, the next cell runs
        Decision d = pick({q(7, 60, 0, true), q(8, 10)}, {r(7, 60, true, true, 1)}, 60, 100, 1, 4);
        CHECK(d.job == 1);
    }
    {   // submission order within a cell: the second request of cell 1 waits
        //   behind the first even if it alone could start
        Decision d = pick({q(1, 500), q(1, 10, 0, true)}, {r(1, 10, false, true, 1)}, 10, 100, 0, 4);
        CHECK(d.job == -1);
    }
    {   // eviction of an idle grid makes room
        Decision d = pick({q(2, 50)}, {r(3, 80, false, false, 1)}, 80, 100, 0, 4);
        CHECK(d.job == 0 && d.evict.size() == 1 && d.evict[0] == 0);
    }
    {   // grids with nothing queued go first, even if more recently used
        std::vector<Resident> res = {r(3, 40, false, true, 1), r(4, 40, false, false, 2)};
        Decision d = pick({q(2, 50), q(3, 40, 0, true)}, res, 80, 100, 0, 4);
        CHECK(d.job == 0 && d.evict.size() == 1 && d.evict[0] == 1);
    }
    {   // least recently used first among equals
        std::vector<Resident> res = {r(3, 40, false, false, 5), r(4, 40, false, false, 2)};
        Decision d = pick({q(2, 50)}, res, 80, 100, 0, 4);
        CHECK(d.job == 0 && d.evict.size() == 1 && d.evict[0] == 1);
    }
    {   // busy grids are never evicted; the blocked request holds later new-memory
        //   requests (no overtaking), but a resident reuse still starts
        std::vector<Resident> res = {r(5, 80, true, false, 1), r(6, 10, false, true, 2)};
        Decision d = pick({q(2, 50), q(9, 5), q(6, 10, 1, true)}, res, 90, 100, 1, 4);
        CHECK(d.job == 2 && d.evict.empty());
        Decision d2 = pick({q(2, 50), q(9, 5)}, res, 90, 100, 1, 4);
        CHECK(d2.job == -1);
    }
    {   // a resident grid of another shape for the same cell is replaced
        Decision d = pick({q(1, 30, 0, false)}, {r(1, 40, false, true, 1)}, 90, 100, 0, 4);
        CHECK(d.job == 0 && d.evict.size() == 1 && d.evict[0] == 0);
    }
    {   // evicting everything idle is still not enough: wait
        Decision d = pick({q(2, 95)}, {r(5, 50, true, false, 1), r(6, 40, false, false, 2)}, 90, 100,
                          1, 4);
        CHECK(d.job == -1);
    }
    {   // percentiles (nearest rank)
        std::vector<double> v;
        for (int i = 100; i >= 1; --i) v.push_back(i);
        CHECK(percentile(v, 50) == 50);
        CHECK(percentile(v, 99) == 99);
        CHECK(percentile(v, 100) == 100);
        CHECK(percentile({5.0}, 99) == 5.0);
        CHECK(percentile({}, 50) == 0.0);
    }
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
