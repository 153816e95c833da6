// Autotuner state: the recorded tile per (family, workload) and the
// per-thread forcing used while candidates are timed.
#include "tune.h"

#include <cstdio>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

namespace harpia {

namespace {

std::mutex g_mu;
std::unordered_map<uint64_t, Tile> g_table;

thread_local int t_forced_fam = -1;
thread_local Tile t_forced;
thread_local std::vector<uint64_t> t_seen;

constexpr int kVolumeRanges[] = {0, 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
constexpr int kBatchZ[] = {0, 8, 16, 32, 64, 128, 256};
constexpr int kBoxXY[][2] = {{64, 8}, {64, 4}, {32, 8}, {32, 4}, {128, 4}};
constexpr int kBoxZ[] = {32, 64, 128, 256};

bool is_volume(int fam) { return fam == TF_GAUSS || fam == TF_GAUSS_DOT || fam == TF_GRAY || fam == TF_BINARY; }
bool is_box(int fam) { return fam == TF_ARGEXT_BOX || fam == TF_GATHER_BOX; }

// FNV-1a over 64-bit words.
struct Hash {
    uint64_t h = 1469598103934665603ull;
    void add(uint64_t v)
    {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    }
};

}  // namespace

const char *tune_family_name(int fam)
{
    static const char *names[TF_COUNT] = {"gauss",         "gauss_dot",         "gray",        "binary",
                                          "gauss_batched", "gauss_dot_batched", "gray_batched", "argext_box",
                                          "gather_box"};
    return fam >= 0 && fam < TF_COUNT ? names[fam] : "?";
}

int tune_candidates(int fam)
{
    if (is_volume(fam)) return (int)(sizeof(kVolumeRanges) / sizeof(int));
    if (is_box(fam)) return 1 + (int)(sizeof(kBoxXY) / sizeof(kBoxXY[0]) * (sizeof(kBoxZ) / sizeof(int)));
    if (fam >= 0 && fam < TF_COUNT) return (int)(sizeof(kBatchZ) / sizeof(int));
    return 0;
}

Tile tune_candidate(int fam, int i)
{
    Tile t;
    if (i <= 0 || i >= tune_candidates(fam)) return t;
    if (is_volume(fam)) {
        t.tz = kVolumeRanges[i];
    } else if (is_box(fam)) {
        const int nz = (int)(sizeof(kBoxZ) / sizeof(int));
        t.tx = kBoxXY[(i - 1) / nz][0];
        t.ty = kBoxXY[(i - 1) / nz][1];
        t.tz = kBoxZ[(i - 1) % nz];
    } else {
        t.tz = kBatchZ[i];
    }
    return t;
}

uint64_t tune_key_volume(int fam, int r, int type_code, const int64_t ext[3])
{
    Hash h;
    h.add((uint64_t)fam);
    h.add((uint64_t)r);
    h.add((uint64_t)type_code);
    for (int i = 0; i < 3; ++i) h.add((uint64_t)ext[i]);
    return h.h;
}

uint64_t tune_key_batch(int fam, int r, int type_code, const BatchDesc &d)
{
    Hash h;
    h.add((uint64_t)fam | 0x100);
    h.add((uint64_t)r);
    h.add((uint64_t)type_code);
    h.add((uint64_t)d.n_crops);
    for (int c = 0; c < d.n_crops; ++c)
        for (int i = 0; i < 3; ++i) h.add((uint64_t)d.c[c].n[i]);
    return h.h;
}

bool tune_lookup(int fam, uint64_t key, Tile &t)
{
    if (t_forced_fam == fam) {
        t_seen.push_back(key);
        t = t_forced;
        return t.tx != 0 || t.ty != 0 || t.tz != 0;
    }
    std::lock_guard<std::mutex> g(g_mu);
    const auto it = g_table.find(key);
    if (it == g_table.end()) return false;
    t = it->second;
    return true;
}

void tune_force(int fam, int i)
{
    if (i < 0) {
        t_forced_fam = -1;
        return;
    }
    t_forced_fam = fam;
    t_forced = tune_candidate(fam, i);
    t_seen.clear();
}

void tune_record_seen(int fam, const Tile &t)
{
    (void)fam;
    std::lock_guard<std::mutex> g(g_mu);
    for (const uint64_t k : t_seen) {
        if (t.tx == 0 && t.ty == 0 && t.tz == 0)
            g_table.erase(k);
        else
            g_table[k] = t;
    }
    t_seen.clear();
}

void tune_clear()
{
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
}

int64_t tune_size()
{
    std::lock_guard<std::mutex> g(g_mu);
    return (int64_t)g_table.size();
}

bool tune_save(const char *path)
{
    std::lock_guard<std::mutex> g(g_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return false;
    std::fprintf(f, "harpia-tune 1\n");
    for (const auto &kv : g_table)
        std::fprintf(f, "%016llx %d %d %d\n", (unsigned long long)kv.first, kv.second.tx, kv.second.ty, kv.second.tz);
    return std::fclose(f) == 0;
}

bool tune_load(const char *path)
{
    // every line after the header must hold exactly "key tx ty tz"
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    std::vector<std::pair<uint64_t, Tile>> rows;
    char line[256];
    bool ok = std::fgets(line, sizeof(line), f) && std::string(line) == "harpia-tune 1\n";
    while (ok && std::fgets(line, sizeof(line), f)) {
        if (line[0] == '\n') continue;
        unsigned long long k;
        Tile t;
        char extra;
        ok = std::sscanf(line, "%llx %d %d %d %c", &k, &t.tx, &t.ty, &t.tz, &extra) == 4;
        if (ok) rows.emplace_back((uint64_t)k, t);
    }
    std::fclose(f);
    if (!ok) return false;
    std::lock_guard<std::mutex> g(g_mu);
    for (const auto &kv : rows) g_table[kv.first] = kv.second;
    return true;
}

}  // namespace harpia
