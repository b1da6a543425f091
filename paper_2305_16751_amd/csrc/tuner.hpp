// Tile choices of the kernels and their cache.  The tuner itself (timing the
// candidates on a plan's own records) lives with the plan code; this header
// holds the choice, its defaults and the persistent cache keyed by
// (device, record kind, record key bits, ceil(log2 E)); the device is its
// architecture name and compute-unit count, e.g. "gfx950:sramecc+:xnack-/256".
//
// Cache file: $DOM_AGG_TUNE_CACHE, else $HOME/.cache/dom_agg_tune.txt; one
// line per key: "device kind key_bits log2E record_sort_tile scan_items
// digit_bits" (lines of any other shape are ignored).
// DOM_AGG_TUNE=0 disables tuning (defaults are used).
#pragma once

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

namespace domagg {

struct TuneChoice {
    int record_sort_tile = 4096;  // onesweep tile: 2048 (256 x 8), 4096 (256 x 16), 8192 (512 x 16) or 16384 (512 x 32)
    int point_sort_tile = 8192;
    int scan_items = 16;          // segmented-scan tile = 256 * items (8 forced for 64-bit keys)
    int digit_bits = 8;           // record-sort digit width: 8, or 7 (tiles 4096 and 8192 only)
};

inline bool valid_sort_tile(int t) { return t == 2048 || t == 4096 || t == 8192 || t == 16384; }

inline TuneChoice default_tune() { return TuneChoice{}; }

using TuneKey = std::tuple<std::string, int, int, int>;

class TuneCache {
  public:
    static TuneCache &get() {
        static TuneCache c;
        return c;
    }
    bool enabled() const {
        const char *e = std::getenv("DOM_AGG_TUNE");
        return !(e && e[0] == '0');
    }
    bool lookup(const TuneKey &k, TuneChoice *out) {
        std::lock_guard<std::mutex> lk(mu_);
        load_once();
        auto it = map_.find(k);
        if (it == map_.end()) return false;
        *out = it->second;
        return true;
    }
    void store(const TuneKey &k, const TuneChoice &c) {
        std::lock_guard<std::mutex> lk(mu_);
        load_once();
        map_[k] = c;
        const std::string p = path();
        if (p.empty()) return;
        if (FILE *f = std::fopen(p.c_str(), "w")) {
            for (auto &kv : map_)
                std::fprintf(f, "%s %d %d %d %d %d %d\n", std::get<0>(kv.first).c_str(), std::get<1>(kv.first),
                             std::get<2>(kv.first), std::get<3>(kv.first), kv.second.record_sort_tile,
                             kv.second.scan_items, kv.second.digit_bits);
            std::fclose(f);
        }
    }

  private:
    std::string path() const {
        if (const char *e = std::getenv("DOM_AGG_TUNE_CACHE")) return e;
        const char *h = std::getenv("HOME");
        if (!h) return "";
        return std::string(h) + "/.cache/dom_agg_tune.txt";
    }
    void load_once() {
        if (loaded_) return;
        loaded_ = true;
        const std::string p = path();
        if (p.empty()) return;
        FILE *f = std::fopen(p.c_str(), "r");
        if (!f) return;
        char line[512], dev[256];
        while (std::fgets(line, sizeof line, f)) {
            int m, kb, le, rs, sc, db;
            if (std::sscanf(line, "%255s %d %d %d %d %d %d", dev, &m, &kb, &le, &rs, &sc, &db) != 7) continue;
            if (!valid_sort_tile(rs) || (sc != 8 && sc != 16) || (db != 7 && db != 8)) continue;
            if (db == 7 && rs != 4096 && rs != 8192) continue;
            TuneChoice c;
            c.record_sort_tile = rs;
            c.scan_items = sc;
            c.digit_bits = db;
            map_[TuneKey{dev, m, kb, le}] = c;
        }
        std::fclose(f);
    }
    std::mutex mu_;
    bool loaded_ = false;
    std::map<TuneKey, TuneChoice> map_;
};

}  // namespace domagg
