// Admission of serving batches by device bytes (host code only, no device
// calls, so that it can be tested on its own): the byte layout of a batch
// and a first-fit allocator of regions of one device allocation.
#pragma once

#include <cstdint>
#include <map>

namespace rambo_pool {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kNone = ~0ull;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Offsets (from the start of the batch's region) of what a batch of n_reads
// reads and n_bytes read bytes keeps on the device, and its size: the read
// count and n_reads + 1 offsets, the read bytes, and the per-read state of
// the query kernels (state_bytes for n_reads reads: the group masks of every
// repetition and the window counts, from which the K-bit answers are
// written straight to host memory).
struct BatchLayout {
    uint64_t hdr = 0, chars = 0, state = 0, total = 0;
};

inline BatchLayout batch_layout(uint64_t n_reads, uint64_t n_bytes, uint64_t state_bytes)
{
    BatchLayout l;
    l.hdr = 0;
    l.chars = l.hdr + align_up(8 * (n_reads + 2));
    l.state = l.chars + align_up(n_bytes);
    l.total = l.state + align_up(state_bytes);
    return l;
}

// One queued request as batch formation sees it: its reads and read
// bytes, or a barrier (an insert) that no batch may pass.
struct Queued {
    bool barrier = false;
    uint64_t reads = 0, bytes = 0;
};

// How many of the n_queued requests at the head of the queue the next batch
// takes, in order: as many as keep it within max_reads reads, max_bytes
// read bytes and `room` device bytes (need(reads, bytes): the device bytes
// of a batch), and, past its first request, within `share` device bytes
// (so that one batch does not take all the room other slots could run
// in).  reads and bytes receive the batch's totals.  0 when the head is a
// barrier or does not fit on its own (it waits for room).
template <class At, class Need>
size_t batch_take(size_t n_queued, At at, Need need, uint64_t max_reads, uint64_t max_bytes, uint64_t room,
                  uint64_t share, uint64_t &reads, uint64_t &bytes)
{
    reads = bytes = 0;
    size_t n = 0;
    for (; n < n_queued; ++n) {
        const Queued q = at(n);
        if (q.barrier || reads + q.reads > max_reads || bytes + q.bytes > max_bytes)
            break;
        const uint64_t b = need(reads + q.reads, bytes + q.bytes);
        if (b > room || (n > 0 && b > share))
            break;
        reads += q.reads;
        bytes += q.bytes;
    }
    return n;
}

// First-fit allocation of kAlign-multiple regions of [0, size); freed
// regions merge with free neighbours.
class Pool {
public:
    explicit Pool(uint64_t size = 0) { reset(size); }

    void reset(uint64_t size)
    {
        size_ = size / kAlign * kAlign;
        free_.clear();
        if (size_)
            free_[0] = size_;
        used_ = peak_ = 0;
    }

    // Start of a free region of `bytes` (rounded up to kAlign), or kNone.
    uint64_t alloc(uint64_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes)
                continue;
            const uint64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes)
                free_[off + bytes] = len - bytes;
            used_ += bytes;
            if (used_ > peak_)
                peak_ = used_;
            return off;
        }
        return kNone;
    }

    // Give back a region that alloc returned for the same `bytes`.
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        uint64_t start = off, len = bytes;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
    }

    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (const auto &f : free_)
            m = f.second > m ? f.second : m;
        return m;
    }

    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    size_t free_blocks() const { return free_.size(); }

private:
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;   // start -> length, no two adjacent
};

}  // namespace rambo_pool
