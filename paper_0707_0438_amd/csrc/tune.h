// Launch-shape cache of the autotuner: the fastest (tile_j, ipt, wg, split)
// measured for a precision and a shape bucket (floor log2 of the i and j
// counts) on one GPU architecture, kept in memory and optionally in a text
// file of one JSON object per line.
#pragma once

#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "nbody.h"

namespace nb {

inline int log2_bucket(int64_t n) {
    int b = 0;
    while (n > 1) {
        n >>= 1;
        ++b;
    }
    return b;
}

class TuneCache {
  public:
    struct Entry {
        int prec, bi, bj;
        nbody_tile t;
        double ms;
    };

    void set_path(const char* p) { path_ = p ? p : ""; }
    void set_arch(const char* a) {
        arch_ = a ? a : "";
        const size_t colon = arch_.find(':');
        if (colon != std::string::npos) arch_.resize(colon);
    }
    const std::string& path() const { return path_; }

    bool lookup(int prec, int64_t ni, int64_t nj, nbody_tile* out) const {
        const int bi = log2_bucket(ni), bj = log2_bucket(nj);
        for (const Entry& e : entries_)
            if (e.prec == prec && e.bi == bi && e.bj == bj) {
                *out = e.t;
                return true;
            }
        return false;
    }

    void store(int prec, int64_t ni, int64_t nj, const nbody_tile& t, double ms) {
        const int bi = log2_bucket(ni), bj = log2_bucket(nj);
        for (Entry& e : entries_)
            if (e.prec == prec && e.bi == bi && e.bj == bj) {
                e.t = t;
                e.ms = ms;
                return;
            }
        entries_.push_back(Entry{prec, bi, bj, t, ms});
    }

    // Lines look like
    // {"arch": "gfx950", "prec": 1, "ni_log2": 20, "nj_log2": 20, "tile_j": 128, "ipt": 2, "wg": 256,
    //  "split": 1, "jsrc": 0, "unroll": 0, "waves": 0, "ms": 812.5}   (one line)
    void load() {
        if (path_.empty()) return;
        FILE* f = fopen(path_.c_str(), "r");
        if (!f) return;
        char line[512];
        while (fgets(line, sizeof line, f)) {
            char arch[64] = {0};
            Entry e{};
            const int got = sscanf(line,
                                   " {\"arch\": \"%63[^\"]\", \"prec\": %d, \"ni_log2\": %d, \"nj_log2\": %d, "
                                   "\"tile_j\": %d, \"ipt\": %d, \"wg\": %d, \"split\": %d, \"jsrc\": %d, "
                                   "\"unroll\": %d, \"waves\": %d, \"ms\": %lf",
                                   arch, &e.prec, &e.bi, &e.bj, &e.t.tile_j, &e.t.ipt, &e.t.wg, &e.t.split, &e.t.jsrc,
                                   &e.t.unroll, &e.t.waves, &e.ms);
            if (got == 12 && arch_ == arch) store_entry(e);
        }
        fclose(f);
    }

    bool save() const {
        if (path_.empty()) return true;
        const std::string tmp = path_ + ".tmp";
        FILE* f = fopen(tmp.c_str(), "w");
        if (!f) return false;
        for (const Entry& e : entries_)
            fprintf(f,
                    "{\"arch\": \"%s\", \"prec\": %d, \"ni_log2\": %d, \"nj_log2\": %d, \"tile_j\": %d, "
                    "\"ipt\": %d, \"wg\": %d, \"split\": %d, \"jsrc\": %d, \"unroll\": %d, \"waves\": %d, "
                    "\"ms\": %.6f}\n",
                    arch_.c_str(), e.prec, e.bi, e.bj, e.t.tile_j, e.t.ipt, e.t.wg, e.t.split, e.t.jsrc, e.t.unroll,
                    e.t.waves, e.ms);
        fclose(f);
        return rename(tmp.c_str(), path_.c_str()) == 0;
    }

  private:
    void store_entry(const Entry& e) {
        for (Entry& x : entries_)
            if (x.prec == e.prec && x.bi == e.bi && x.bj == e.bj) {
                x = e;
                return;
            }
        entries_.push_back(e);
    }
    std::string path_, arch_;
    std::vector<Entry> entries_;
};

}  // namespace nb
