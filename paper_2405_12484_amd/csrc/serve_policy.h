// Scheduling policy of the step-request server: which garments wait for
// device memory, which frames go into the next launch, and request latency.
// Pure host logic (no HIP), so it can be exercised on its own.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace vh {

struct ServeRequest {
    uint64_t ticket = 0;
    int32_t garment = -1;
    int32_t frames = 0;     // frames requested
    int32_t launched = 0;   // frames handed to a launch
    int32_t done = 0;       // frames completed
    double t_arrival = 0.0, t_done = -1.0;
};

class ServePolicy {
  public:
    enum State { QUEUED = 0, RESIDENT = 1, RELEASED = 2 };

    int32_t add_garment() {
        gs_.push_back(Garment());
        fifo_.push_back((int32_t)gs_.size() - 1);
        return (int32_t)gs_.size() - 1;
    }
    int32_t n_garments() const { return (int32_t)gs_.size(); }
    State state(int32_t g) const { return gs_[g].state; }

    // Queued garments in admission (FIFO) order.
    std::vector<int32_t> queued() const {
        std::vector<int32_t> q;
        for (int32_t g : fifo_)
            if (gs_[g].state == QUEUED) q.push_back(g);
        return q;
    }

    // Device bytes garment g takes once admitted.
    void set_need(int32_t g, size_t bytes) { gs_[g].need = bytes; }
    size_t need(int32_t g) const { return gs_[g].need; }

    // The queued garments to admit now, in FIFO order, with `in_use` bytes held
    // and `budget` bytes in all (0 = unlimited): strictly first come, first
    // served, so admission stops at the first garment that does not fit.
    std::vector<int32_t> to_admit(size_t in_use, size_t budget) const {
        std::vector<int32_t> out;
        for (int32_t g : queued()) {
            if (budget && in_use + gs_[g].need > budget) break;
            in_use += gs_[g].need;
            out.push_back(g);
        }
        return out;
    }
    void admit(int32_t g) { gs_[g].state = RESIDENT; }
    void release(int32_t g) { gs_[g].state = RELEASED; }

    uint64_t submit(int32_t g, int32_t frames, double t) {
        ServeRequest r;
        r.ticket = reqs_.size() + 1;
        r.garment = g;
        r.frames = frames;
        r.t_arrival = t;
        reqs_.push_back(r);
        gs_[g].pending.push_back(r.ticket);
        if (t < t_first_) t_first_ = t;
        return r.ticket;
    }

    // Resident garments with a frame not yet handed to a launch, ordered by the
    // arrival of the request that frame belongs to (ties: garment id), at most
    // max_garments of them.  A garment may have frames in several queued
    // launches: launches on one stream run in order.
    std::vector<int32_t> pick(int32_t max_garments) const {
        std::vector<std::pair<double, int32_t>> c;
        for (int32_t g = 0; g < (int32_t)gs_.size(); ++g) {
            const Garment& G = gs_[g];
            if (G.state != RESIDENT) continue;
            const ServeRequest* r = next_unlaunched(G);
            if (r) c.push_back({r->t_arrival, g});
        }
        std::sort(c.begin(), c.end());
        std::vector<int32_t> out;
        for (size_t i = 0; i < c.size() && (int32_t)i < max_garments; ++i) out.push_back(c[i].second);
        return out;
    }

    // One frame of each garment handed to a launch.
    void launch(const std::vector<int32_t>& gs) {
        for (int32_t g : gs) {
            Garment& G = gs_[g];
            ServeRequest& r = reqs_[next_unlaunched(G)->ticket - 1];
            r.launched++;
            G.in_flight++;
        }
    }

    // The oldest launched frame of each garment finished at time t.
    void complete(const std::vector<int32_t>& gs, double t) {
        for (int32_t g : gs) {
            Garment& G = gs_[g];
            ServeRequest& r = reqs_[G.pending.front() - 1];
            r.done++;
            frames_done_++;
            G.in_flight--;
            if (r.done == r.frames) {
                r.t_done = t;
                lat_.push_back(t - r.t_arrival);
                G.pending.pop_front();
                if (t > t_last_) t_last_ = t;
            }
        }
    }

    bool idle(int32_t g) const { return gs_[g].in_flight == 0 && gs_[g].pending.empty(); }
    int32_t in_flight(int32_t g) const { return gs_[g].in_flight; }
    bool any_pending() const {
        for (const Garment& G : gs_)
            if (G.state != RELEASED && (!G.pending.empty() || G.in_flight > 0)) return true;
        return false;
    }
    const ServeRequest* find(uint64_t ticket) const {
        return (ticket >= 1 && ticket <= reqs_.size()) ? &reqs_[ticket - 1] : nullptr;
    }

    // Forget completed requests' latencies and the throughput window (queued
    // and running requests are kept).
    void reset_stats() {
        lat_.clear();
        frames_done_ = 0;
        t_first_ = 1e300;
        t_last_ = -1e300;
        for (const Garment& G : gs_)
            for (uint64_t t : G.pending) t_first_ = std::min(t_first_, reqs_[t - 1].t_arrival);
    }

    int64_t frames_done() const { return frames_done_; }
    int64_t requests_done() const { return (int64_t)lat_.size(); }
    double span() const { return (t_last_ > t_first_) ? t_last_ - t_first_ : 0.0; }
    // q-quantile (nearest rank) of the completed requests' latencies
    double percentile(double q) const {
        if (lat_.empty()) return 0.0;
        std::vector<double> v = lat_;
        std::sort(v.begin(), v.end());
        size_t k = (size_t)std::max(0.0, std::min((double)v.size() - 1.0, q * (double)v.size() - 1e-9));
        return v[k];
    }

  private:
    struct Garment {
        State state = QUEUED;
        std::deque<uint64_t> pending;   // requests not yet completed, FIFO
        int32_t in_flight = 0;          // frames launched, not yet completed
        size_t need = 0;                // device bytes once admitted
    };
    const ServeRequest* next_unlaunched(const Garment& G) const {
        for (uint64_t t : G.pending) {
            const ServeRequest& r = reqs_[t - 1];
            if (r.launched < r.frames) return &r;
        }
        return nullptr;
    }
    std::vector<Garment> gs_;
    std::vector<int32_t> fifo_;
    std::vector<ServeRequest> reqs_;
    std::vector<double> lat_;
    int64_t frames_done_ = 0;
    double t_first_ = 1e300, t_last_ = -1e300;
};

}  // namespace vh
