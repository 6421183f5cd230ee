// fft3d_arena.hpp -- sub-allocation of one device region (the server's HBM
// budget): best fit over free blocks, neighbours merged on free.  Host-side
// bookkeeping only; offsets are relative to the region.
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>

namespace fft3d {

class Arena {
public:
    static constexpr size_t kAlign = 256;

    void reset(size_t bytes)
    {
        size_ = bytes & ~(kAlign - 1);
        by_off_.clear();
        by_len_.clear();
        used_ = 0;
        if (size_) insert(0, size_);
    }

    // Offset of a new block of `bytes` (rounded up to kAlign), or false.
    bool alloc(size_t bytes, size_t* off)
    {
        const size_t n = round(bytes);
        auto it = by_len_.lower_bound(n);
        if (it == by_len_.end()) return false;
        const size_t len = it->first, at = it->second;
        erase(at, len);
        if (len > n) insert(at + n, len - n);
        used_ += n;
        *off = at;
        return true;
    }

    void free(size_t off, size_t bytes)
    {
        size_t n = round(bytes), at = off;
        used_ -= n;
        auto next = by_off_.lower_bound(at);
        if (next != by_off_.end() && next->first == at + n) {  // merge with the block after
            n += next->second;
            erase(next->first, next->second);
        }
        auto prev = by_off_.lower_bound(at);
        if (prev != by_off_.begin()) {
            prev = std::prev(prev);
            if (prev->first + prev->second == at) {  // ... and the one before
                at = prev->first;
                n += prev->second;
                erase(prev->first, prev->second);
            }
        }
        insert(at, n);
    }

    static size_t round(size_t bytes) { return (bytes + kAlign - 1) & ~(kAlign - 1); }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t largest_free() const { return by_len_.empty() ? 0 : by_len_.rbegin()->first; }
    size_t free_blocks() const { return by_off_.size(); }

private:
    void insert(size_t off, size_t len)
    {
        by_off_[off] = len;
        by_len_.emplace(len, off);
    }
    void erase(size_t off, size_t len)
    {
        by_off_.erase(off);
        auto r = by_len_.equal_range(len);
        for (auto it = r.first; it != r.second; ++it)
            if (it->second == off) {
                by_len_.erase(it);
                break;
            }
    }

    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> by_off_;       // free blocks by offset
    std::multimap<size_t, size_t> by_len_;  // the same by length
};

}  // namespace fft3d
