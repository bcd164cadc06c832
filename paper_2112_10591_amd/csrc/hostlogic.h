// hostlogic.h -- host-only pieces of the runtime that need no GPU: the
// first-fit arena sub-allocator, the FIFO byte ring used for event staging,
// and the rule that forms a served batch.  Kept free of HIP so that they can
// be unit-tested on the CPU.
#pragma once

#include <cerrno>
#include <climits>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <deque>
#include <iterator>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace ebof {

// First-fit sub-allocator over a caller-owned address range (bookkeeping
// only; it never touches the memory).  Blocks are 256-byte aligned and sized.
class Arena {
   public:
    void init(char* base, size_t size) {
        base_ = base;
        size_ = size;
        used_ = 0;
        free_.clear();
        inuse_.clear();
        if (size) free_[0] = size;
    }
    void* alloc(size_t bytes, size_t align = 256) {
        if (bytes == 0) bytes = 1;
        bytes = (bytes + 255) & ~size_t(255);
        if (align < 256) align = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const size_t off = it->first, sz = it->second;
            const size_t aoff = (off + align - 1) / align * align;
            if (aoff + bytes <= off + sz) {
                free_.erase(it);
                if (aoff > off) free_[off] = aoff - off;
                if (off + sz > aoff + bytes) free_[aoff + bytes] = off + sz - (aoff + bytes);
                inuse_[aoff] = bytes;
                used_ += bytes;
                return base_ + aoff;
            }
        }
        return nullptr;
    }
    void free(void* p) {
        if (!p) return;
        size_t off = (size_t)((char*)p - base_);
        auto it = inuse_.find(off);
        if (it == inuse_.end()) return;
        size_t sz = it->second;
        inuse_.erase(it);
        used_ -= sz;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + sz == nx->first) {
            sz += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += sz;
                return;
            }
        }
        free_[off] = sz;
    }
    size_t bytes_free() const { return size_ - used_; }
    size_t bytes_used() const { return used_; }
    size_t free_blocks() const { return free_.size(); }

   private:
    char* base_ = nullptr;
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    std::map<size_t, size_t> inuse_;  // offset -> size
};

// FIFO ring of byte ranges: ranges are allocated in order, released in any
// order, and space is reclaimed from the oldest live range on.
class Ring {
   public:
    void init(size_t size) {
        size_ = size;
        head_ = 0;
        live_.clear();
    }
    bool alloc(size_t len, size_t* off) {
        len = (len ? len + 255 : 256) & ~size_t(255);
        if (len > size_) return false;
        size_t o;
        if (live_.empty()) {
            o = 0;
        } else {
            const size_t front = live_.front().off;
            if (head_ > front) {  // not wrapped: free space is [head, size) and [0, front)
                if (head_ + len <= size_)
                    o = head_;
                else if (len <= front)
                    o = 0;
                else
                    return false;
            } else {  // wrapped: free space is [head, front)
                if (head_ + len <= front)
                    o = head_;
                else
                    return false;
            }
        }
        live_.push_back({o, len, false});
        head_ = o + len;
        *off = o;
        return true;
    }
    void release(size_t off) {
        for (auto& s : live_)
            if (s.off == off && !s.done) {
                s.done = true;
                break;
            }
        while (!live_.empty() && live_.front().done) live_.pop_front();
        if (live_.empty()) head_ = 0;
    }
    size_t live() const { return live_.size(); }

   private:
    struct Seg {
        size_t off, len;
        bool done;
    };
    size_t size_ = 0, head_ = 0;
    std::deque<Seg> live_;
};

// Served batch formation: walk the queue in submission order and take at
// most one window per stream (a stream's next window needs this one's
// pyramid), up to max_n windows; the rest stays queued in order.
template <class T, class SidOf>
std::vector<T> take_one_per_stream(std::deque<T>& queue, int max_n, SidOf sid_of) {
    std::vector<T> take;
    std::set<int32_t> used;
    for (auto it = queue.begin(); it != queue.end() && (int)take.size() < max_n;) {
        const int32_t sid = sid_of(*it);
        if (used.count(sid)) {
            ++it;
            continue;
        }
        used.insert(sid);
        take.push_back(*it);
        it = queue.erase(it);
    }
    return take;
}

// One line of the launch-shape cache: "<key>\t<v_0> <v_1> ... <v_{n-1}>"
// (exactly n integers after the tab; trailing CR/LF ignored).  False for a
// line of any other form.
inline bool parse_tune_line(const std::string& line, int n, std::string* key, std::vector<int>* vals) {
    std::string l = line;
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    const size_t tab = l.find('\t');
    if (tab == std::string::npos || tab == 0) return false;
    std::vector<int> v;
    const char* q = l.c_str() + tab + 1;
    for (int i = 0; i < n; ++i) {
        char* end = nullptr;
        errno = 0;
        const long x = std::strtol(q, &end, 10);
        if (end == q || errno || x < INT32_MIN || x > INT32_MAX) return false;
        v.push_back((int)x);
        q = end;
    }
    while (*q == ' ') ++q;
    if (*q) return false;
    *key = l.substr(0, tab);
    *vals = v;
    return true;
}

}  // namespace ebof
