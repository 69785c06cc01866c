// Host-side bookkeeping of a context's simulations (no HIP dependency, so
// the logic is also compiled and tested on its own on the CPU).
//
//  - live: every simulation created on the context and not yet destroyed.
//    Destroying the context destroys what is still live, so no simulation
//    handle can outlive the context it points into.
//  - pending: the simulations advanced by a launch that can abort (the
//    persistent sweeps wait for neighbours with a bounded wait) since the
//    last synchronising call checked the context's abort flag.  The flag is
//    sticky: once raised it stays raised until a synchronising call reads it;
//    that call then marks every pending simulation invalid and clears the
//    flag, so an abort cannot be lost to a later launch that finished cleanly.
#pragma once
#include <algorithm>
#include <vector>

namespace fskmc {

template <class Sim>
class SimRegistry {
  public:
    void add(Sim* s) { live_.push_back(s); }

    // A simulation leaves both lists when it is destroyed.
    void remove(Sim* s)
    {
        live_.erase(std::remove(live_.begin(), live_.end(), s), live_.end());
        pending_.erase(std::remove(pending_.begin(), pending_.end(), s), pending_.end());
    }

    // Called when a launch that can abort has been enqueued for s.
    void touched(Sim* s)
    {
        if (std::find(pending_.begin(), pending_.end(), s) == pending_.end())
            pending_.push_back(s);
    }

    // After a synchronisation: the simulations whose lattices an abort left
    // unspecified (all pending ones when the flag was raised), and the
    // pending list starts over.
    std::vector<Sim*> settle(bool aborted)
    {
        std::vector<Sim*> hit;
        if (aborted)
            hit.swap(pending_);
        pending_.clear();
        return hit;
    }

    // The live simulations, handed over for destruction with the context.
    std::vector<Sim*> release_all()
    {
        std::vector<Sim*> all;
        all.swap(live_);
        pending_.clear();
        return all;
    }

    size_t n_live() const { return live_.size(); }
    size_t n_pending() const { return pending_.size(); }
    bool is_live(const Sim* s) const { return std::find(live_.begin(), live_.end(), s) != live_.end(); }

  private:
    std::vector<Sim*> live_;
    std::vector<Sim*> pending_;
};

}  // namespace fskmc
