// Host-policy checks (no GPU): admission accounting of the request server and
// the bounded cache of the convenience entry points.  Prints one line per
// check and exits non-zero on the first failure.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "bed_admit.hpp"
#include "bed_lru.hpp"

static int g_fail = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond); \
            g_fail = 1;                                               \
        }                                                             \
    } while (0)

static void admission()
{
    using namespace bed;
    CHECK(request_bytes(3, 4, 4) == 3 * (2 * 16 + 4) * 4);
    Admission a;
    a.max_mats = 10;
    CHECK(a.admit(6, 100) == ADMIT_OK);
    CHECK(a.admit(5, 100) == ADMIT_INFLIGHT);  // 6 + 5 > 10
    CHECK(a.mats == 6 && a.bytes == 100);      // a refusal changes nothing
    CHECK(a.admit(4, 100) == ADMIT_OK);        // exactly at the limit
    CHECK(a.admit(1, 1) == ADMIT_INFLIGHT);
    a.release(6, 100);
    CHECK(a.admit(1, 1) == ADMIT_OK);
    a.release(4, 100);
    a.release(1, 1);
    CHECK(a.idle() && a.bytes == 0);

    Admission m;
    m.max_bytes = 1000;
    CHECK(m.admit(1, 600) == ADMIT_OK);
    CHECK(m.admit(1, 401) == ADMIT_MEMORY);
    CHECK(m.admit(1, 400) == ADMIT_OK);
    CHECK(m.admit(1000000, 0) == ADMIT_OK);  // no matrix limit
    Admission tiny;
    tiny.max_bytes = 64;
    CHECK(tiny.admit(1, request_bytes(1, 8, 4)) == ADMIT_MEMORY);
    Admission none;
    CHECK(none.admit(1 << 30, int64_t(1) << 50) == ADMIT_OK);  // 0 = unlimited
    std::printf("admission ok\n");
}

static void lru()
{
    bed::Lru<int, std::string> c(3);
    CHECK(c.insert(1, "a").empty());
    CHECK(c.insert(2, "b").empty());
    CHECK(c.insert(3, "c").empty());
    CHECK(c.size() == 3 && c.capacity() == 3);
    CHECK(c.find(1) && *c.find(1) == "a");  // 1 becomes most recent: 2 is oldest
    auto ev = c.insert(4, "d");
    CHECK(ev.size() == 1 && ev[0] == "b");
    CHECK(!c.find(2) && c.size() == 3);
    c.pin(3);                 // pinned entries are never evicted
    CHECK(c.find(1) != nullptr);
    ev = c.insert(5, "e");    // oldest unpinned is 4 (3 is pinned)
    CHECK(ev.size() == 1 && ev[0] == "d");
    c.pin(1);
    c.pin(5);
    ev = c.insert(6, "f");    // everything pinned: grows past capacity
    CHECK(ev.empty() && c.size() == 4);
    CHECK(c.find(3) && c.find(6));
    // many distinct keys: size stays at capacity once unpinned entries cycle
    bed::Lru<int, int> d(8);
    size_t evicted = 0;
    for (int k = 0; k < 1000; ++k) evicted += d.insert(k, k).size();
    CHECK(d.size() == 8 && evicted == 992);
    for (int k = 992; k < 1000; ++k) CHECK(d.find(k) && *d.find(k) == k);
    std::printf("lru ok\n");
}

int main()
{
    admission();
    lru();
    return g_fail;
}
