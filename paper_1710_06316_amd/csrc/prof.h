// Per-phase timing with HIP events on the stream each phase runs on.
#pragma once
#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace afmpb {

struct Prof {
    bool on = false;
    std::string only;   // non-empty: time only the scopes of this name
    struct Entry {
        std::string name;
        double ms = 0;
        long long count = 0;
    };
    std::vector<Entry> entries;
    std::map<std::string, int> index;
    // (entry, start, stop) events awaiting readout
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> pool;
    int open = 0;   // scopes not yet closed (pending is only flushed at zero)
    int id_of(const char *name);
    hipEvent_t take();
    void flush();   // synchronises on pending events and accumulates
    ~Prof();
};

}  // namespace afmpb
