// elastic.hpp - bookkeeping of an address range whose physical memory is committed in
// granules only where slots are in use (pure host code, no HIP calls; api.hip maps and
// unmaps the runs it returns).
//
// A slot owns byte ranges [off, off + len) of the range; ranges of different slots never
// overlap but may share a granule at their ends. Granules entirely inside one slot's
// range form one run, committed and released with the slot; a granule a range covers
// only in part may be shared with the neighbouring slot and is committed on its own,
// reference-counted, and released with its last user. So every committed run is
// released whole, exactly as it was committed.
#pragma once
#include <cstddef>
#include <vector>

namespace sapdd {

struct GranRun {
    size_t g, n;  // first granule, granules
};

class ElasticPlan {
  public:
    ElasticPlan() = default;
    ElasticPlan(size_t granule, size_t bytes) : gran_(granule), refs_((bytes + granule - 1) / granule, 0) {}
    size_t granule() const { return gran_; }
    size_t granules() const { return refs_.size(); }
    size_t committed() const { return committed_; }  // granules currently committed

    // Reference [off, off + len); appends the runs to commit now to `out`.
    void acquire(size_t off, size_t len, std::vector<GranRun> &out) {
        if (len == 0) return;
        size_t i0, i1, b[2];
        int nb = split(off, len, i0, i1, b);
        if (i1 > i0) {  // exclusive interior: committed as one run
            for (size_t g = i0; g < i1; ++g) refs_[g] = 1;
            out.push_back({i0, i1 - i0});
            committed_ += i1 - i0;
        }
        for (int k = 0; k < nb; ++k)
            if (refs_[b[k]]++ == 0) {
                out.push_back({b[k], 1});
                committed_ += 1;
            }
    }
    // Drop the reference of [off, off + len); appends the runs to release now to `out`.
    void release(size_t off, size_t len, std::vector<GranRun> &out) {
        if (len == 0) return;
        size_t i0, i1, b[2];
        int nb = split(off, len, i0, i1, b);
        if (i1 > i0) {
            for (size_t g = i0; g < i1; ++g) refs_[g] = 0;
            out.push_back({i0, i1 - i0});
            committed_ -= i1 - i0;
        }
        for (int k = 0; k < nb; ++k)
            if (--refs_[b[k]] == 0) {
                out.push_back({b[k], 1});
                committed_ -= 1;
            }
    }
    // Granules an acquire of a range of len bytes can commit at most.
    size_t max_granules(size_t len) const { return len == 0 ? 0 : (len + gran_ - 1) / gran_ + 1; }
    int refs(size_t g) const { return refs_[g]; }

  private:
    // interior granules [i0, i1) lie wholly inside the range; b[0..nb) are the (at most
    // two) granules it covers in part
    int split(size_t off, size_t len, size_t &i0, size_t &i1, size_t b[2]) const {
        const size_t end = off + len;
        const size_t g0 = off / gran_, g1 = (end + gran_ - 1) / gran_;
        i0 = (off + gran_ - 1) / gran_;
        i1 = end / gran_;
        if (i1 < i0) i1 = i0;  // the range lies inside one granule
        int nb = 0;
        for (size_t g = g0; g < g1; ++g)
            if (g < i0 || g >= i1) b[nb++] = g;
        return nb;
    }
    size_t gran_ = 1;
    std::vector<int> refs_;
    size_t committed_ = 0;
};

}  // namespace sapdd
