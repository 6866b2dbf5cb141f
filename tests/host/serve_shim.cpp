// Test-only C entry points over the step server's scheduling policy
// (paper_2405_12484_amd/csrc/serve_policy.h), so that admission, request
// ordering and latency bookkeeping can be driven from a CPU test with a
// synthetic clock.
#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../paper_2405_12484_amd/csrc/serve_policy.h"

using vh::ServePolicy;

extern "C" {

void* vhp_pol_new() { return new ServePolicy(); }
void vhp_pol_free(void* p) { delete static_cast<ServePolicy*>(p); }

int vhp_pol_add(void* p, size_t need) {
    ServePolicy& P = *static_cast<ServePolicy*>(p);
    const int g = P.add_garment();
    P.set_need(g, need);
    return g;
}

int vhp_pol_state(void* p, int g) { return static_cast<ServePolicy*>(p)->state(g); }

int vhp_pol_to_admit(void* p, size_t in_use, size_t budget, int* out, int cap) {
    std::vector<int32_t> v = static_cast<ServePolicy*>(p)->to_admit(in_use, budget);
    int n = 0;
    for (int32_t g : v)
        if (n < cap) out[n++] = g;
    return (int)v.size();
}

void vhp_pol_admit(void* p, int g) { static_cast<ServePolicy*>(p)->admit(g); }
void vhp_pol_release(void* p, int g) { static_cast<ServePolicy*>(p)->release(g); }

uint64_t vhp_pol_submit(void* p, int g, int frames, double t) {
    return static_cast<ServePolicy*>(p)->submit(g, frames, t);
}

int vhp_pol_pick(void* p, int max_garments, int* out, int cap) {
    std::vector<int32_t> v = static_cast<ServePolicy*>(p)->pick(max_garments);
    int n = 0;
    for (int32_t g : v)
        if (n < cap) out[n++] = g;
    return (int)v.size();
}

void vhp_pol_launch(void* p, const int* ids, int n) {
    static_cast<ServePolicy*>(p)->launch(std::vector<int32_t>(ids, ids + n));
}

void vhp_pol_complete(void* p, const int* ids, int n, double t) {
    static_cast<ServePolicy*>(p)->complete(std::vector<int32_t>(ids, ids + n), t);
}

int vhp_pol_idle(void* p, int g) { return static_cast<ServePolicy*>(p)->idle(g) ? 1 : 0; }
int vhp_pol_in_flight(void* p, int g) { return static_cast<ServePolicy*>(p)->in_flight(g); }
int vhp_pol_any_pending(void* p) { return static_cast<ServePolicy*>(p)->any_pending() ? 1 : 0; }

// launched, done, garment of a request; returns 0 if the ticket is unknown
int vhp_pol_request(void* p, uint64_t ticket, int* launched, int* done, int* garment, double* t_done) {
    const vh::ServeRequest* r = static_cast<ServePolicy*>(p)->find(ticket);
    if (!r) return 0;
    *launched = r->launched;
    *done = r->done;
    *garment = r->garment;
    *t_done = r->t_done;
    return 1;
}

double vhp_pol_percentile(void* p, double q) { return static_cast<ServePolicy*>(p)->percentile(q); }
double vhp_pol_span(void* p) { return static_cast<ServePolicy*>(p)->span(); }
int64_t vhp_pol_frames_done(void* p) { return static_cast<ServePolicy*>(p)->frames_done(); }
int64_t vhp_pol_requests_done(void* p) { return static_cast<ServePolicy*>(p)->requests_done(); }

}  // extern "C"
