// Placement of request texts in the serving loop's device byte ring (host
// logic only: no device calls, so it is tested on its own on the CPU).
//
// Occupied bytes are [head, tail) when the ring is not wrapped, else
// [head, size) + [0, tail).  A request that does not fit before the end of
// the ring starts at 0 and also holds the unused end bytes until it is
// released.  Requests are released in the order they were placed; the bytes
// they hold, their own plus such end bytes, never exceed the budget.
#pragma once

#include <cstdint>

namespace pfac {

class TextRing {
public:
    struct Span {
        uint64_t off = 0;    // first byte of the text
        uint64_t n = 0;      // text bytes
        uint64_t len = 0;    // bytes held: the text and any unused end bytes
        bool wraps = false;  // placed at 0, holding the end bytes
    };

    TextRing(uint64_t size, uint64_t budget) : size_(size), budget_(budget) {}

    // Where n bytes would go now (off), and how many unused end bytes they
    // would hold with them (pad).  False when they do not fit.
    bool fits(uint64_t n, uint64_t &off, uint64_t &pad) const {
        if (n > size_) return false;
        if (!wrapped_) {
            if (size_ - tail_ >= n) {
                off = tail_;
                pad = 0;
            } else if (head_ >= n) {
                off = 0;
                pad = size_ - tail_;
            } else {
                return false;
            }
        } else {
            if (head_ - tail_ < n) return false;
            off = tail_;
            pad = 0;
        }
        return used_ + n + pad <= budget_;
    }

    // Take the place fits() chose; `empty` = no placed span is held.
    Span place(uint64_t n, uint64_t off, uint64_t pad, bool empty) {
        Span s;
        s.off = off;
        s.n = n;
        s.len = n + pad;
        s.wraps = !wrapped_ && off == 0 && !empty;
        if (s.wraps) wrapped_ = true;
        tail_ = off + n;
        used_ += s.len;
        return s;
    }

    // Release the oldest held span; `empty` = it was the last one.
    void release(const Span &s, bool empty) {
        used_ -= s.len;
        if (s.wraps) wrapped_ = false;
        head_ = s.off + s.n;
        if (empty) {
            head_ = tail_ = used_ = 0;
            wrapped_ = false;
        }
    }

    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }

private:
    uint64_t size_ = 0, budget_ = 0;
    uint64_t head_ = 0, tail_ = 0, used_ = 0;
    bool wrapped_ = false;
};

}  // namespace pfac
