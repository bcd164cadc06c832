// Host-only checks of the runtime's allocator, staging ring and served-batch
// rule (no GPU).  Built and run by tests/test_host_logic.py.
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <string>
#include <set>
#include <utility>
#include <vector>

#include "../../paper_2112_10591_amd/csrc/hostlogic.h"

using namespace ebof;

static uint64_t rng_state = 12345;
static uint64_t rnd() {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return rng_state >> 33;
}

static bool overlaps(const std::map<size_t, size_t>& live, size_t off, size_t len) {
    for (auto& kv : live)
        if (off < kv.first + kv.second && kv.first < off + len) return true;
    return false;
}

static void test_arena() {
    static char base_mem[1];
    char* base = base_mem;  // bookkeeping only: never dereferenced
    Arena a;
    a.init(base, 1 << 20);
    assert(a.bytes_free() == (1u << 20));
    void* p = a.alloc(100);
    void* q = a.alloc(300);
    assert(p == base && (char*)q == base + 256);  // 256-byte rounding
    assert(a.bytes_used() == 256 + 512);
    assert(a.alloc(1 << 21) == nullptr);          // larger than the arena
    a.free(p);
    void* r = a.alloc(200);                        // first fit reuses the hole
    assert(r == base);
    a.free(q);
    a.free(r);
    assert(a.bytes_used() == 0 && a.free_blocks() == 1);  // fully coalesced
    // random stress against an interval model
    std::map<size_t, size_t> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rnd() % 3) {
            size_t len = 1 + rnd() % 20000;
            char* x = (char*)a.alloc(len);
            if (!x) continue;
            size_t off = x - base;
            size_t rl = (len + 255) & ~size_t(255);
            assert(off % 256 == 0 && off + rl <= (1u << 20));
            assert(!overlaps(live, off, rl));
            live[off] = rl;
        } else {
            auto it2 = live.begin();
            std::advance(it2, rnd() % live.size());
            a.free(base + it2->first);
            live.erase(it2);
        }
        size_t used = 0;
        for (auto& kv : live) used += kv.second;
        assert(used == a.bytes_used());
    }
    for (auto& kv : live) a.free(base + kv.first);
    assert(a.bytes_used() == 0 && a.free_blocks() == 1);
}

static void test_ring() {
    Ring r;
    r.init(4096);
    size_t o1, o2, o3, o4;
    assert(r.alloc(1000, &o1) && o1 == 0);
    assert(r.alloc(1000, &o2) && o2 == 1024);
    assert(r.alloc(1000, &o3) && o3 == 2048);
    assert(!r.alloc(2000, &o4));       // only 1024 left at the end, front busy
    r.release(o2);                     // out of order: nothing reclaimed yet
    assert(!r.alloc(1500, &o4));
    r.release(o1);                     // front released: [0, 2048) free again
    assert(r.alloc(1500, &o4) && o4 == 0);  // wraps to the start
    assert(!r.alloc(5000, &o4));       // larger than the ring
    r.release(o3);
    r.release(0);
    assert(r.live() == 0);
    // random stress: live ranges never overlap and stay inside the ring
    Ring s;
    s.init(1 << 16);
    std::map<size_t, size_t> live;
    std::deque<size_t> order;
    for (int it = 0; it < 50000; ++it) {
        if (order.empty() || rnd() % 2) {
            size_t len = 1 + rnd() % 9000, off;
            if (s.alloc(len, &off)) {
                size_t rl = (len + 255) & ~size_t(255);
                assert(off + rl <= (1u << 16));
                assert(!overlaps(live, off, rl));
                live[off] = rl;
                order.push_back(off);
            }
        } else {
            size_t k = rnd() % order.size();
            s.release(order[k]);
            live.erase(order[k]);
            order.erase(order.begin() + k);
        }
    }
}

struct W {
    int sid, id;
};

static void test_take_one_per_stream() {
    std::deque<W> q = {{1, 0}, {2, 1}, {1, 2}, {3, 3}, {2, 4}, {4, 5}, {1, 6}};
    auto t = take_one_per_stream(q, 3, [](const W& w) { return w.sid; });
    assert(t.size() == 3 && t[0].id == 0 && t[1].id == 1 && t[2].id == 3);
    assert(q.size() == 4 && q[0].id == 2 && q[1].id == 4 && q[2].id == 5 && q[3].id == 6);
    auto t2 = take_one_per_stream(q, 10, [](const W& w) { return w.sid; });
    assert(t2.size() == 3 && t2[0].id == 2 && t2[1].id == 4 && t2[2].id == 5);
    assert(q.size() == 1 && q[0].id == 6);
    // every window of a stream is taken in submission order over successive batches
    std::deque<W> big;
    for (int i = 0; i < 1000; ++i) big.push_back({(int)(rnd() % 17), i});
    std::map<int, int> last;
    while (!big.empty()) {
        auto b = take_one_per_stream(big, 5, [](const W& w) { return w.sid; });
        std::set<int> seen;
        for (auto& w : b) {
            assert(seen.insert(w.sid).second);
            assert(!last.count(w.sid) || last[w.sid] < w.id);
            last[w.sid] = w.id;
        }
    }
}

#define CHECK(c) do { if (!(c)) { std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); std::abort(); } } while (0)

static void test_parse_tune_line() {
    std::string key;
    std::vector<int> v;
    CHECK(ebof::parse_tune_line("1280,720,4,4,1,0;\t4 64 0 2048 -1\n", 5, &key, &v));
    CHECK(key == "1280,720,4,4,1,0;" && v.size() == 5 && v[0] == 4 && v[2] == 0 && v[4] == -1);
    CHECK(ebof::parse_tune_line("k\t1 2 3 \r\n", 3, &key, &v));
    CHECK(!ebof::parse_tune_line("k\t1 2", 3, &key, &v));          // too few
    CHECK(!ebof::parse_tune_line("k\t1 2 3 4", 3, &key, &v));      // too many
    CHECK(!ebof::parse_tune_line("k 1 2 3", 3, &key, &v));          // no tab
    CHECK(!ebof::parse_tune_line("\t1 2 3", 3, &key, &v));         // empty key
    CHECK(!ebof::parse_tune_line("k\t1 x 3", 3, &key, &v));        // not a number
    CHECK(!ebof::parse_tune_line("k\t1 99999999999 3", 3, &key, &v));  // out of range
}

int main() {
    test_parse_tune_line();
    test_arena();
    test_ring();
    test_take_one_per_stream();
    std::puts("hostlogic ok");
    return 0;
}
