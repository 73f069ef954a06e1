// tune.cpp -- lookup of the tile shape chosen by the autotuner.
//
// Table format (text, one rule per line, '#' comments):
//   prec  m_max  n_max  tile
// The first rule with prec equal and m <= m_max and n <= n_max wins.
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "corr2d_internal.h"
#include "tune.h"

namespace corr2d {
namespace {

struct Rule {
    int prec;
    int64_t m_max, n_max;
    int tile;
};

std::once_flag g_once;
std::vector<Rule> g_rules;
std::string g_source = "no table: size rule";

std::string default_path() {
    Dl_info info;
    if (dladdr((void*)&tune_lookup, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        const size_t slash = p.find_last_of('/');
        const std::string dir = slash == std::string::npos ? "." : p.substr(0, slash);
        return dir + "/tune/gfx950.tsv";
    }
    return "tune/gfx950.tsv";
}

void load() {
    const char* env = std::getenv("CORR2D_TUNE_TABLE");
    const std::string path = env && *env ? std::string(env) : default_path();
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        Rule r;
        long long mm, nn;
        if (std::sscanf(line, "%d %lld %lld %d", &r.prec, &mm, &nn, &r.tile) == 4) {
            r.m_max = mm;
            r.n_max = nn;
            if (r.tile >= 1 && r.tile <= 3) g_rules.push_back(r);
        }
    }
    std::fclose(f);
    g_source = path + " (" + std::to_string(g_rules.size()) + " rules)";
}

}  // namespace

const char* tune_source() {
    std::call_once(g_once, load);
    return g_source.c_str();
}

int tune_lookup(int prec, int64_t m, int64_t n) {
    std::call_once(g_once, load);
    for (const Rule& r : g_rules)
        if (r.prec == prec && m <= r.m_max && n <= r.n_max) {
            if (prec == P_F64 && r.tile != 1 && r.tile != 2) continue;
            if (blocked_layout(prec) && r.tile != 2 && r.tile != 3) continue;
            if (!blocked_layout(prec) && r.tile == 3) continue;
            return r.tile;
        }
    if (prec == P_F64) return 1;
    if (blocked_layout(prec)) return 3;
    return n <= 1024 ? 1 : 2;
}

}  // namespace corr2d
