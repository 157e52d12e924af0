// Tile-shape autotuner of the compositing passes (host code): times a
// caller-supplied training step for each candidate (tile shape, wavefronts
// per tile in the forward and in the backward) with HIP events on the
// caller's stream, keeps the fastest per workload key, and caches the
// choices in memory and, when a cache file is set, in a JSON file of the
// form {"<key>": {"tile": [w, h, fwd, bwd], "ms": {"WxHxFxB": ms, ...}}}.
#include <cctype>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gs_internal.hpp"

namespace gs {
namespace {

struct TuneEntry {
    gs_tune_choice best{};
    std::vector<std::pair<std::string, double>> ms;   // candidate label -> ms per step
};

std::mutex g_tune_mu;
std::string g_tune_path;                     // empty: memory only
std::map<std::string, TuneEntry> g_tune;     // key -> entry (memory and file contents)
bool g_tune_loaded = false;

// ---- minimal JSON reader for the cache file (objects, arrays, strings,
// numbers, true/false/null); unknown fields are skipped

struct Json {
    const char* p;
    const char* e;
    bool ok = true;

    void ws() {
        while (p < e && std::isspace(static_cast<unsigned char>(*p))) p++;
    }
    bool eat(char c) {
        ws();
        if (p < e && *p == c) {
            p++;
            return true;
        }
        return false;
    }
    bool str(std::string& out) {
        ws();
        if (p >= e || *p != '"') return ok = false;
        p++;
        out.clear();
        while (p < e && *p != '"') {
            if (*p == '\\' && p + 1 < e) {
                p++;
                const char c = *p;
                out.push_back(c == 'n' ? '\n' : (c == 't' ? '\t' : c));
            } else {
                out.push_back(*p);
            }
            p++;
        }
        if (p >= e) return ok = false;
        p++;
        return true;
    }
    bool num(double& v) {
        ws();
        char* end = nullptr;
        v = std::strtod(p, &end);
        if (end == p || end > e) return ok = false;
        p = end;
        return true;
    }
    void skip() {   // any value
        ws();
        if (p >= e) {
            ok = false;
            return;
        }
        if (*p == '"') {
            std::string s;
            str(s);
        } else if (*p == '{') {
            p++;
            if (eat('}')) return;
            do {
                std::string k;
                if (!str(k) || !eat(':')) {
                    ok = false;
                    return;
                }
                skip();
            } while (ok && eat(','));
            if (!eat('}')) ok = false;
        } else if (*p == '[') {
            p++;
            if (eat(']')) return;
            do skip();
            while (ok && eat(','));
            if (!eat(']')) ok = false;
        } else if (std::strncmp(p, "true", 4) == 0) {
            p += 4;
        } else if (std::strncmp(p, "false", 5) == 0) {
            p += 5;
        } else if (std::strncmp(p, "null", 4) == 0) {
            p += 4;
        } else {
            double v;
            num(v);
        }
    }
};

// parses one cache entry {"tile": [..4 ints..], "ms": {...}, ...}
bool parse_entry(Json& j, TuneEntry& out) {
    if (!j.eat('{')) return false;
    bool have_tile = false;
    if (j.eat('}')) return false;
    do {
        std::string k;
        if (!j.str(k) || !j.eat(':')) return false;
        if (k == "tile") {
            if (!j.eat('[')) return false;
            double v[4];
            for (int i = 0; i < 4; i++) {
                if (i && !j.eat(',')) return false;
                if (!j.num(v[i])) return false;
            }
            if (!j.eat(']')) return false;
            out.best.tile_w = int32_t(v[0]);
            out.best.tile_h = int32_t(v[1]);
            out.best.fwd_waves = int32_t(v[2]);
            out.best.bwd_waves = int32_t(v[3]);
            have_tile = true;
        } else if (k == "ms") {
            if (!j.eat('{')) return false;
            if (!j.eat('}')) {
                do {
                    std::string lab;
                    double v;
                    if (!j.str(lab) || !j.eat(':') || !j.num(v)) return false;
                    out.ms.emplace_back(lab, v);
                } while (j.eat(','));
                if (!j.eat('}')) return false;
            }
        } else {
            j.skip();
        }
        if (!j.ok) return false;
    } while (j.eat(','));
    return j.eat('}') && have_tile;
}

// reads the cache file into g_tune (entries already in memory win); a
// missing file is an empty cache, a malformed one an error
bool load_file(std::string& err) {
    if (g_tune_path.empty()) return true;
    FILE* f = std::fopen(g_tune_path.c_str(), "rb");
    if (!f) return true;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    Json j{text.data(), text.data() + text.size()};
    j.ws();
    if (j.p == j.e) return true;
    if (!j.eat('{')) {
        err = "tune cache " + g_tune_path + ": not a JSON object";
        return false;
    }
    if (j.eat('}')) return true;
    do {
        std::string key;
        TuneEntry ent;
        if (!j.str(key) || !j.eat(':') || !parse_entry(j, ent)) {
            err = "tune cache " + g_tune_path + ": malformed entry";
            return false;
        }
        g_tune.emplace(key, ent);
    } while (j.eat(','));
    if (!j.eat('}')) {
        err = "tune cache " + g_tune_path + ": malformed";
        return false;
    }
    return true;
}

void put_str(std::string& o, const std::string& s) {
    o.push_back('"');
    for (char c : s) {
        if (c == '"' || c == '\\') o.push_back('\\');
        o.push_back(c);
    }
    o.push_back('"');
}

bool save_file(std::string& err) {
    if (g_tune_path.empty()) return true;
    std::string o = "{\n";
    bool first = true;
    char num[64];
    for (const auto& kv : g_tune) {
        if (!first) o += ",\n";
        first = false;
        o += " ";
        put_str(o, kv.first);
        const gs_tune_choice& b = kv.second.best;
        std::snprintf(num, sizeof num, ": {\"tile\": [%d, %d, %d, %d], \"ms\": {", int(b.tile_w), int(b.tile_h),
                      int(b.fwd_waves), int(b.bwd_waves));
        o += num;
        bool f2 = true;
        for (const auto& m : kv.second.ms) {
            if (!f2) o += ", ";
            f2 = false;
            put_str(o, m.first);
            std::snprintf(num, sizeof num, ": %.6g", m.second);
            o += num;
        }
        o += "}}";
    }
    o += "\n}\n";
    const std::string tmp = g_tune_path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) {
        err = "cannot write " + tmp;
        return false;
    }
    const bool wrote = std::fwrite(o.data(), 1, o.size(), f) == o.size();
    if (std::fclose(f) != 0 || !wrote || std::rename(tmp.c_str(), g_tune_path.c_str()) != 0) {
        err = "cannot write " + g_tune_path;
        return false;
    }
    return true;
}

std::string label(const gs_tune_choice& c) {
    char b[64];
    std::snprintf(b, sizeof b, "%dx%dx%dx%d", int(c.tile_w), int(c.tile_h), int(c.fwd_waves), int(c.bwd_waves));
    return b;
}

}  // namespace

gs_status tune_set_cache(const char* path, std::string& err) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_path = path ? path : "";
    g_tune_loaded = true;
    return load_file(err) ? GS_OK : GS_E_INVALID;
}

gs_status tune_lookup(const char* key, gs_tune_choice* best, double* best_ms, bool* found, std::string& err) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        if (!load_file(err)) return GS_E_INVALID;
    }
    auto it = g_tune.find(key);
    *found = it != g_tune.end();
    if (*found) {
        *best = it->second.best;
        if (best_ms) {
            *best_ms = -1.0;
            const std::string lab = label(it->second.best);
            for (const auto& m : it->second.ms)
                if (m.first == lab) *best_ms = m.second;
        }
    }
    return GS_OK;
}

gs_status tune_run(const char* key, const gs_tune_choice* cand, int32_t n, int32_t reps, gs_tune_step_fn step,
                   void* user, hipStream_t stream, gs_tune_choice* best, double* best_ms, std::string& err) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        err = "hipEventCreate failed";
        return GS_E_DEVICE;
    }
    TuneEntry ent;
    double best_t = 0.0;
    int best_i = -1;
    gs_status st = GS_OK;
    for (int i = 0; i < n && st == GS_OK; i++) {
        if (step(&cand[i], user) != 0) {   // warm-up, and the caller's buffer sizing
            err = "tune step failed for " + label(cand[i]);
            st = GS_E_INVALID;
            break;
        }
        if (hipStreamSynchronize(stream) != hipSuccess || hipEventRecord(e0, stream) != hipSuccess) {
            err = "stream error while tuning";
            st = GS_E_DEVICE;
            break;
        }
        for (int r = 0; r < reps; r++) {
            if (step(&cand[i], user) != 0) {
                err = "tune step failed for " + label(cand[i]);
                st = GS_E_INVALID;
                break;
            }
        }
        if (st != GS_OK) break;
        float ms = 0.f;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            err = "event timing failed while tuning";
            st = GS_E_DEVICE;
            break;
        }
        const double t = double(ms) / reps;
        ent.ms.emplace_back(label(cand[i]), t);
        if (best_i < 0 || t < best_t) {
            best_t = t;
            best_i = i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GS_OK) return st;
    ent.best = cand[best_i];
    *best = ent.best;
    if (best_ms) *best_ms = best_t;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = ent;
    return save_file(err) ? GS_OK : GS_E_INVALID;
}

}  // namespace gs
