// Autotuner tables of librac: per problem shape (kind of call, domain size,
// variables, constraint density, states per call), the path and work-item
// size measured fastest on this GPU. Entries come from a measurement run on
// the first call of a shape (rac_host.hip runs every candidate on the call's
// own inputs, which give identical results, and keeps the fastest), and are
// kept in a text file so that later processes start from them; a table
// measured on an MI355X ships with the library. Host code only.
#include <dlfcn.h>
#include <sys/stat.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "rac_tune.h"

namespace rac {

namespace {

std::mutex g_mu;
bool g_loaded = false;
std::map<std::string, TuneChoice> g_table;   // key -> choice (user file over shipped table)

int32_t pow2_at_least(int64_t v, int64_t lo) {
    int64_t p = lo;
    while (p < v) p <<= 1;
    return (int32_t)p;
}

const char *density_bucket(double dens) {
    if (dens <= 0.05) return "0.05";
    if (dens <= 0.1) return "0.1";
    if (dens <= 0.25) return "0.25";
    if (dens <= 0.5) return "0.5";
    if (dens <= 0.75) return "0.75";
    return "1";
}

bool parse_line(const char *line, std::string *key, TuneChoice *c) {
    // "<key> path=<p> items=<s> handoff=<h> ms=<t>", key without spaces
    char k[128];
    int p = 0, s = 0, h = 0;
    double ms = 0.0;
    if (sscanf(line, "%127s path=%d items=%d handoff=%d ms=%lf", k, &p, &s, &h, &ms) != 5) return false;
    if (p < 1 || p > 4 || s < -4 || s > 4 || h < -1) return false;
    *key = k;
    c->path = p;
    c->item_scale_log2 = s;
    c->handoff = h;
    c->ms = ms;
    return true;
}

void load_file(const std::string &path, int source) {
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        std::string key;
        TuneChoice c;
        if (!parse_line(line, &key, &c)) continue;
        c.source = source;
        g_table[key] = c;   // later lines (and the user file, read last) win
    }
    fclose(f);
}

}  // namespace

int tune_mode() {
    const char *e = getenv("RAC_TUNE");
    if (!e || !*e) return kTuneAuto;
    if (!strcmp(e, "rules")) return kTuneRules;
    if (!strcmp(e, "measure")) return kTuneMeasure;
    return kTuneAuto;
}

std::string tune_user_file() {
    const char *e = getenv("RAC_TUNE_CACHE");
    if (e && *e) return e;
    const char *home = getenv("HOME");
    return std::string(home && *home ? home : "/tmp") + "/.cache/rac_tune_gfx950.txt";
}

std::string tune_key(int kind, int32_t n, int32_t d, int64_t arcs, int32_t B) {
    const double dens = n > 1 ? (double)arcs / ((double)n * (double)(n - 1)) : 0.0;
    char buf[128];
    snprintf(buf, sizeof(buf), "gfx950/%s/d%d/n%d/dens%s/B%d", kind == kTuneBatch ? "batch" : "single",
             pow2_at_least(d, 4), pow2_at_least(n, 16), density_bucket(dens),
             kind == kTuneBatch ? pow2_at_least(B, 2) : 1);
    return buf;
}

std::string tune_shipped_file() {
    const char *e = getenv("RAC_TUNE_TABLE");
    if (e && *e) return e;
    Dl_info info;
    if (dladdr((const void *)&tune_shipped_file, &info) && info.dli_fname) {
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) +
               "/rac_tune_gfx950.txt";
    }
    return "rac_tune_gfx950.txt";
}

bool tune_lookup(const std::string &key, TuneChoice *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) {
        load_file(tune_shipped_file(), kSourceShipped);
        load_file(tune_user_file(), kSourceCache);
        g_loaded = true;
    }
    auto it = g_table.find(key);
    if (it == g_table.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string &key, const TuneChoice &c) {
    std::lock_guard<std::mutex> lk(g_mu);
    TuneChoice v = c;
    v.source = kSourceCache;   // later calls find it in the user's table
    g_table[key] = v;
    const std::string path = tune_user_file();
    // the directories of the file may not exist yet
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;   // an unwritable cache only costs a measurement per process
    fprintf(f, "%s path=%d items=%d handoff=%d ms=%.4f\n", key.c_str(), c.path, c.item_scale_log2,
            c.handoff, c.ms);
    fclose(f);
}

void tune_forget() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    g_loaded = false;
}

}  // namespace rac
