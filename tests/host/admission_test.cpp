// CPU test of the serving loop's host admission (admission.hpp): the pool
// allocator against a reference model (a bitmap of 256-byte units with
// first-fit over maximal free runs), and the in-order admission rule with fake
// requests.  Prints one line per failed check and exits non-zero if any.
#include "admission.hpp"

#include <cstdio>
#include <deque>
#include <random>
#include <vector>

using heston::rt::Pool;
using heston::rt::admit_in_order;

static int fails = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);                      \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

// Reference: unit i is used iff used[i]; an allocation takes the lowest
// maximal free run long enough.
struct Ref {
    std::vector<char> used;
    explicit Ref(size_t units) : used(units, 0) {}
    long alloc(size_t units)
    {
        size_t i = 0;
        while (i < used.size()) {
            if (used[i]) {
                ++i;
                continue;
            }
            size_t j = i;
            while (j < used.size() && !used[j])
                ++j;
            if (j - i >= units) {
                for (size_t k = i; k < i + units; ++k)
                    used[k] = 1;
                return (long)i;
            }
            i = j;
        }
        return -1;
    }
    void release(size_t start, size_t units)
    {
        for (size_t k = start; k < start + units; ++k)
            used[k] = 0;
    }
    size_t free_units() const
    {
        size_t n = 0;
        for (char u : used)
            n += !u;
        return n;
    }
};

static void pool_against_reference(unsigned seed)
{
    const size_t units = 1000;
    std::vector<unsigned char> buf(units * 256 + 100); // the tail below 256 B is unusable
    Pool pool;
    pool.init(buf.data(), buf.size());
    Ref ref(units);
    CHECK(pool.free_bytes() == units * 256);
    struct Live {
        unsigned char *p;
        size_t start, units;
    };
    std::vector<Live> live;
    std::mt19937 rng(seed);
    for (int op = 0; op < 20000; ++op) {
        if (live.empty() || rng() % 100 < 55) {
            const size_t bytes = 1 + rng() % 4000;
            const size_t u = (bytes + 255) / 256;
            unsigned char *p = pool.alloc(bytes);
            const long r = ref.alloc(u);
            CHECK((p == nullptr) == (r < 0));
            if (p && r >= 0) {
                CHECK((size_t)(p - buf.data()) == (size_t)r * 256);
                live.push_back({p, (size_t)r, u});
            }
        } else {
            const size_t k = rng() % live.size();
            pool.release(live[k].p);
            ref.release(live[k].start, live[k].units);
            live[k] = live.back();
            live.pop_back();
        }
        CHECK(pool.free_bytes() == ref.free_units() * 256);
        if (fails > 10)
            return;
    }
    for (auto &l : live)
        pool.release(l.p);
    // released neighbours coalesce: the whole pool is one block again
    CHECK(pool.free_bytes() == units * 256);
    unsigned char *all = pool.alloc(units * 256);
    CHECK(all == buf.data());
    CHECK(pool.alloc(1) == nullptr);
    pool.release(all);
    pool.release(all); // a second release of the same block is ignored
    CHECK(pool.free_bytes() == units * 256);
}

static void small_pool_and_reinit()
{
    std::vector<unsigned char> buf(4096);
    Pool pool;
    pool.init(buf.data(), 200);
    CHECK(pool.free_bytes() == 0);
    CHECK(pool.alloc(1) == nullptr);
    pool.init(buf.data(), 4096);
    unsigned char *a = pool.alloc(1000);
    CHECK(a == buf.data());
    pool.init(buf.data(), 4096); // forgets every allocation
    CHECK(pool.free_bytes() == 4096);
    CHECK(pool.alloc(4096) == buf.data());
}

struct FakeReq {
    int id;
    uint64_t bytes;
    unsigned char *mem = nullptr;
};

static void admission_rule()
{
    std::vector<unsigned char> buf(10 * 256);
    Pool pool;
    pool.init(buf.data(), buf.size());
    std::vector<FakeReq> reqs = {{0, 4 * 256}, {1, 4 * 256}, {2, 3 * 256}, {3, 256}, {4, 256}};
    std::deque<FakeReq *> queue;
    std::vector<FakeReq *> active;
    for (auto &r : reqs)
        queue.push_back(&r);
    auto bytes = [](const FakeReq *q) { return q->bytes; };
    auto place = [](FakeReq *q, unsigned char *m) { q->mem = m; };
    // 0 and 1 fit (8 of 10 units); 2 needs 3 units and blocks 3 and 4 behind it
    size_t n = admit_in_order(queue, active, 8, pool, bytes, place);
    CHECK(n == 2);
    CHECK(active.size() == 2 && active[0]->id == 0 && active[1]->id == 1);
    CHECK(queue.front()->id == 2);
    CHECK(reqs[0].mem == buf.data() && reqs[1].mem == buf.data() + 4 * 256);
    // releasing 0 lets 2, then 3 in; 4 waits for the slot limit of 4
    pool.release(reqs[0].mem);
    active.erase(active.begin());
    n = admit_in_order(queue, active, 3, pool, bytes, place);
    CHECK(n == 2);
    CHECK(active.size() == 3 && active[1]->id == 2 && active[2]->id == 3);
    CHECK(queue.size() == 1 && queue.front()->id == 4);
    n = admit_in_order(queue, active, 3, pool, bytes, place);
    CHECK(n == 0);
    n = admit_in_order(queue, active, 4, pool, bytes, place);
    CHECK(n == 1 && queue.empty());
    CHECK(admit_in_order(queue, active, 4, pool, bytes, place) == 0);
}

int main()
{
    for (unsigned seed = 1; seed <= 5; ++seed)
        pool_against_reference(seed);
    small_pool_and_reinit();
    admission_rule();
    if (fails) {
        std::printf("%d checks failed\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
