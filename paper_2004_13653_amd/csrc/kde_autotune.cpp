// Tile-shape autotuner: the cache of measured choices (host code only).
//
// The FP32 direct kernels come in three register-block shapes (2 x 2, 4 x 4 and
// 8 x 8 pixels per thread, tiles of 32, 64 and 128 nodes).  Which one is fastest
// depends on the kernel's support against the tile, on the number of points and
// on the grid: small tiles waste fewer evaluations on pixels a compact kernel
// cannot reach and give more workgroups; large blocks amortise each factor over
// more FMAs and, in the batched launch, scan each map's points for fewer tiles.
// kde_api.cpp times the candidates on the caller's own data the first time it
// meets a shape bucket and stores the winner here; later calls in the same
// bucket reuse it.
//
// Keys: "eval/<arch>/<gauss|compact>/H<b>/n<b>/px<b>" for single maps (log2
// buckets of the bandwidth in pixels, the point count and the pixel count) and
// "batch/<arch>/<hash>" for batches (FNV-1a hash of each map's kernel class,
// point count and grid).  Choices: "2", "4" or "8" for single maps, "<g>,<c>"
// (Gaussian maps, compact maps) for batches.
//
// The cache persists as JSON:
//   {"format": "kde-autotune-1",
//    "entries": {"<key>": {"choice": "<choice>", "ms": {"<candidate>": <ms>, ...}}, ...}}
// A file that does not parse, has another format tag or holds an invalid choice
// is rejected as a whole (and the cache keeps its previous content), so a corrupt
// or foreign cache only costs a re-tune.
#include "kde_internal.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace kde {
namespace tune {

namespace {

constexpr const char *kFormat = "kde-autotune-1";

struct State {
    std::mutex mu;
    std::map<std::string, Entry> entries;
    bool init = false;
    bool enabled = true;
    int forced = 0;
    std::string path;  // KDE_AUTOTUNE_CACHE: loaded at first use, saved after each new entry
};

State &state() {
    static State s;
    return s;
}

// ------------------------------------------------------------ JSON subset
// Objects, strings (escapes \" \\ \/ only) and numbers: what save() writes.
struct Parser {
    const char *p, *e;
    bool ok = true;

    void ws() {
        while (p < e && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool eat(char c) {
        ws();
        if (p < e && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string *out) {
        ws();
        if (p >= e || *p != '"') return false;
        ++p;
        out->clear();
        while (p < e && *p != '"') {
            char c = *p++;
            if (c == '\\') {
                if (p >= e) return false;
                c = *p++;
                if (c != '"' && c != '\\' && c != '/') return false;
            } else if ((unsigned char)c < 0x20) {
                return false;
            }
            out->push_back(c);
        }
        if (p >= e) return false;
        ++p;
        return true;
    }
    bool num(double *out) {
        ws();
        const char *b = p;
        while (p < e && (std::strchr("+-0123456789.eE", *p) != nullptr)) ++p;
        if (p == b) return false;
        const std::string t(b, p);
        char *end = nullptr;
        *out = std::strtod(t.c_str(), &end);
        return end == t.c_str() + t.size() && std::isfinite(*out);
    }
    // Calls f(key) for every member of an object; f parses the value.
    template <class F>
    bool object(F f) {
        if (!eat('{')) return false;
        if (eat('}')) return true;
        do {
            std::string k;
            if (!str(&k) || !eat(':') || !f(k)) return false;
        } while (eat(','));
        return eat('}');
    }
};

bool parse_entry(Parser &P, Entry *en) {
    bool have_choice = false;
    const bool ok = P.object([&](const std::string &k) {
        if (k == "choice") return have_choice = P.str(&en->choice);
        if (k == "ms")
            return P.object([&](const std::string &cand) {
                double v = 0.0;
                if (!P.num(&v)) return false;
                en->ms.emplace_back(cand, v);
                return true;
            });
        return false;
    });
    return ok && have_choice;
}

bool parse_file(const std::string &text, std::map<std::string, Entry> *out, std::string *err) {
    Parser P{text.data(), text.data() + text.size()};
    bool have_format = false;
    std::map<std::string, Entry> got;
    const bool ok = P.object([&](const std::string &k) {
        if (k == "format") {
            std::string f;
            if (!P.str(&f) || f != kFormat) return false;
            return have_format = true;
        }
        if (k == "entries")
            return P.object([&](const std::string &key) {
                Entry en;
                if (!parse_entry(P, &en) || !valid_choice(key, en.choice)) return false;
                got[key] = en;
                return true;
            });
        return false;
    });
    P.ws();
    if (!ok || !have_format || P.p != P.e) {
        *err = "not a kde-autotune-1 cache (or a malformed entry)";
        return false;
    }
    *out = std::move(got);
    return true;
}

void put_string(std::string *o, const std::string &s) {
    o->push_back('"');
    for (char c : s) {
        if (c == '"' || c == '\\') o->push_back('\\');
        o->push_back(c);
    }
    o->push_back('"');
}

std::string to_json(const std::map<std::string, Entry> &m) {
    std::string o = "{\"format\": \"";
    o += kFormat;
    o += "\",\n \"entries\": {";
    bool first = true;
    for (const auto &kv : m) {
        o += first ? "\n  " : ",\n  ";
        first = false;
        put_string(&o, kv.first);
        o += ": {\"choice\": ";
        put_string(&o, kv.second.choice);
        o += ", \"ms\": {";
        for (size_t i = 0; i < kv.second.ms.size(); ++i) {
            if (i) o += ", ";
            put_string(&o, kv.second.ms[i].first);
            char buf[64];
            std::snprintf(buf, sizeof buf, ": %.6g", kv.second.ms[i].second);
            o += buf;
        }
        o += "}}";
    }
    o += "}}\n";
    return o;
}

bool read_text(const char *path, std::string *text) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    char buf[4096];
    size_t k;
    text->clear();
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) {
        text->append(buf, k);
        if (text->size() > (size_t(64) << 20)) break;  // no cache is this large
    }
    std::fclose(f);
    return true;
}

bool write_text(const std::string &path, const std::string &text, std::string *err) {
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) {
        *err = "cannot open " + tmp + " for writing";
        return false;
    }
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    if (std::fclose(f) != 0 || !ok) {
        std::remove(tmp.c_str());
        *err = "cannot write " + tmp;
        return false;
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        *err = "cannot rename " + tmp + " to " + path;
        return false;
    }
    return true;
}

// Reads the environment once: KDE_AUTOTUNE=0 switches tuning off, KDE_TILE=2|4|8
// forces a shape, KDE_AUTOTUNE_CACHE names the persistent cache.
void init_locked(State &s) {
    if (s.init) return;
    s.init = true;
    if (const char *v = std::getenv("KDE_AUTOTUNE")) s.enabled = std::strcmp(v, "0") != 0;
    if (const char *v = std::getenv("KDE_TILE")) {
        const int rc = std::atoi(v);
        if (valid_rc(rc)) s.forced = rc;
    }
    if (const char *v = std::getenv("KDE_AUTOTUNE_CACHE")) {
        s.path = v;
        std::string text, err;
        std::map<std::string, Entry> got;
        if (!s.path.empty() && read_text(s.path.c_str(), &text) && parse_file(text, &got, &err))
            s.entries = std::move(got);
    }
}

}  // namespace

bool valid_choice(const std::string &key, const std::string &choice) {
    if (key.rfind("eval/", 0) == 0) return choice == "2" || choice == "4" || choice == "8";
    if (key.rfind("batch/", 0) == 0) {
        if (choice.size() != 3 || choice[1] != ',') return false;
        return valid_rc(choice[0] - '0') && valid_rc(choice[2] - '0');
    }
    return false;
}

bool enabled() {
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    return s.enabled;
}

void set_enabled(bool on) {
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    s.enabled = on;
}

int forced() {
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    return s.forced;
}

void set_forced(int rc) {
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    s.forced = rc;
}

bool lookup(const std::string &key, std::string *choice) {
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    auto it = s.entries.find(key);
    if (it == s.entries.end()) return false;
    *choice = it->second.choice;
    return true;
}

void store(const std::string &key, const Entry &e) {
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    s.entries[key] = e;
    if (!s.path.empty()) {
        std::string err;
        (void)write_text(s.path, to_json(s.entries), &err);  // best effort: the in-memory cache stays valid
    }
}

bool load(const char *path, std::string *err) {
    std::string text;
    if (!read_text(path, &text)) {
        *err = std::string("cannot read ") + path;
        return false;
    }
    std::map<std::string, Entry> got;
    if (!parse_file(text, &got, err)) return false;
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    for (auto &kv : got) s.entries[kv.first] = kv.second;
    return true;
}

bool save(const char *path, std::string *err) {
    State &s = state();
    std::string text;
    {
        std::lock_guard<std::mutex> l(s.mu);
        init_locked(s);
        text = to_json(s.entries);
    }
    return write_text(path, text, err);
}

std::string dump() {
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    return to_json(s.entries);
}

void clear() {
    State &s = state();
    std::lock_guard<std::mutex> l(s.mu);
    init_locked(s);
    s.entries.clear();
}

}  // namespace tune
}  // namespace kde
