// tuning.hip -- launch-shape cache: the fused-sweep tile plans and the
// population-annealing workgroup sizes a context holds, written to and read
// back from a small text file, so that tuned shapes outlive the process.
// Launch shapes never change results; only speed.
//
// File format (one entry per line, '#' starts a comment):
//   libmcspin-launch-shapes 1
//   tile <dims> <Lx> <Ly> <Lz> <count> <H> <K> <threads>
//   pa <L> <G>
#include <cerrno>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <tuple>

#include "internal.hpp"

using namespace mcs;

namespace {

constexpr const char *kHeader = "libmcspin-launch-shapes 1";

// the line without its comment and surrounding white space
std::string strip(const char *line)
{
    std::string s(line);
    const size_t hash = s.find('#');
    if (hash != std::string::npos) s.resize(hash);
    const size_t b = s.find_first_not_of(" \t\r\n");
    if (b == std::string::npos) return std::string();
    const size_t e = s.find_last_not_of(" \t\r\n");
    return s.substr(b, e - b + 1);
}

// "<keyword> v0 v1 ... v(n-1)": exactly n decimal integers that fit int32
bool parse_entry(const std::string &s, const char *keyword, int *v, int n)
{
    const size_t kl = std::strlen(keyword);
    if (s.compare(0, kl, keyword) != 0 || (s.size() > kl && s[kl] != ' ' && s[kl] != '\t')) return false;
    const char *p = s.c_str() + kl;
    for (int i = 0; i < n; ++i) {
        while (*p == ' ' || *p == '\t') ++p;
        if (!*p) return false;
        char *end = nullptr;
        errno = 0;
        const long long x = std::strtoll(p, &end, 10);
        if (end == p || errno == ERANGE || x < INT32_MIN || x > INT32_MAX || (*end && *end != ' ' && *end != '\t'))
            return false;
        v[i] = (int)x;
        p = end;
    }
    while (*p == ' ' || *p == '\t') ++p;
    return *p == 0;
}

}  // namespace

extern "C" {

int mc_tuning_save(mc_ctx *ctx, const char *path)
{
    if (!ctx) return MC_E_INVAL;
    if (!path || !*path) return fail(ctx, MC_E_INVAL, "path is NULL or empty");
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(ctx, MC_E_IO, "cannot write %s: %s", tmp.c_str(), std::strerror(errno));
    bool ok = std::fprintf(f, "%s\n", kHeader) > 0;
    for (const auto &kv : ctx->tile_plans) {
        int d, lx, ly, lz, n;
        std::tie(d, lx, ly, lz, n) = kv.first;
        ok = ok && std::fprintf(f, "tile %d %d %d %d %d %d %d %d\n", d, lx, ly, lz, n, kv.second.H, kv.second.K,
                                kv.second.threads) > 0;
    }
    for (const auto &kv : ctx->pa_groups) ok = ok && std::fprintf(f, "pa %d %d\n", kv.first, kv.second) > 0;
    ok = std::fclose(f) == 0 && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(ctx, MC_E_IO, "cannot write %s", path);
    }
    return MC_OK;
}

int mc_tuning_load(mc_ctx *ctx, const char *path)
{
    if (!ctx) return MC_E_INVAL;
    if (!path || !*path) return fail(ctx, MC_E_INVAL, "path is NULL or empty");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(ctx, MC_E_IO, "cannot read %s: %s", path, std::strerror(errno));
    // every entry goes through the setters' checks on a scratch context; the
    // caller's context changes only if the whole file is valid
    mc_ctx scratch;
    scratch.device = ctx->device;
    char line[256];
    int ln = 0, rc = MC_OK;
    bool header = false;
    while (rc == MC_OK && std::fgets(line, sizeof line, f)) {
        ++ln;
        if (!std::strchr(line, '\n') && !std::feof(f)) {
            rc = fail(ctx, MC_E_INVAL, "%s:%d: line too long", path, ln);
            break;
        }
        const std::string s = strip(line);
        if (s.empty()) continue;
        if (!header) {
            if (s != kHeader) rc = fail(ctx, MC_E_INVAL, "%s:%d: not a launch-shape file (expected '%s')", path, ln,
                                        kHeader);
            header = true;
            continue;
        }
        int v[8];
        int r;
        if (parse_entry(s, "tile", v, 8)) {
            const mc_geom g = {v[0], v[1], v[2], v[3], MC_INT8, v[4]};
            r = mc_set_tile_plan(&scratch, &g, v[5], v[6], v[7]);
        } else if (parse_entry(s, "pa", v, 2)) {
            r = v[1] == 0 ? fail(&scratch, MC_E_RANGE, "G = 0 is not a setting") : mc_set_pa_group(&scratch, v[0], v[1]);
        } else {
            r = fail(&scratch, MC_E_INVAL, "unknown entry '%s'", s.c_str());
        }
        if (r) rc = fail(ctx, r, "%s:%d: %s", path, ln, scratch.last_error.c_str());
    }
    if (rc == MC_OK && std::ferror(f)) rc = fail(ctx, MC_E_IO, "cannot read %s", path);
    std::fclose(f);
    if (rc == MC_OK && !header) rc = fail(ctx, MC_E_INVAL, "%s: no header line", path);
    if (rc) return rc;
    for (const auto &kv : scratch.tile_plans) ctx->tile_plans[kv.first] = kv.second;
    for (const auto &kv : scratch.pa_groups) ctx->pa_groups[kv.first] = kv.second;
    return MC_OK;
}

}  // extern "C"
