// Launch autotuner: times the linear search under each number of windows per
// lane and the periodic search under each fold launch shape on the caller's
// own data, keeps the fastest (cetra_set_tuning) and caches it in a JSON file
// keyed by GPU architecture and shape class.  Results of the search do not
// depend on the tuning; only its speed does.
#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace {

using namespace cetra;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int ceil_log2(int64_t v) {
    int k = 0;
    while (((int64_t)1 << k) < v && k < 62) ++k;
    return k;
}

// Work of the timed fold slice: contiguous periods from the middle of the
// grid (neighbouring periods share cache lines as in the full search), about
// 5e11 algorithmic bytes (tens of milliseconds at the fold's rate).
int64_t slice_periods(const cetra_grid *g, int64_t n_periods) {
    const double per_period = 8.0 * g->n_dur * (double)g->n_t0;
    const int64_t n = (int64_t)std::ceil(5.0e11 / std::max(per_period, 1.0));
    return std::max<int64_t>(std::min<int64_t>(n, n_periods), std::min<int64_t>(n_periods, 64));
}

// One cache entry.
struct Entry {
    std::string arch;
    int log2_t0 = 0, n_dur = 0, log2_periods = 0;
    cetra_tuning tu{};
    double fold_ms = 0.0, linear_ms = 0.0;
};

// Reads the entries of a cache file written by write_cache: flat JSON objects
// of "key": number or "key": "string" pairs inside the "entries" array.
// Unknown keys are ignored; a missing or unreadable file has no entries.
std::vector<Entry> read_cache(const char *path) {
    std::vector<Entry> out;
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return out;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, got);
    std::fclose(fp);
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos) return out;
    pos = text.find('[', pos);
    if (pos == std::string::npos) return out;
    while (true) {
        const size_t open = text.find('{', pos);
        const size_t end = text.find(']', pos);
        if (open == std::string::npos || (end != std::string::npos && end < open)) break;
        const size_t close = text.find('}', open);
        if (close == std::string::npos) break;
        Entry e;
        size_t p = open + 1;
        while (p < close) {
            const size_t k0 = text.find('"', p);
            if (k0 == std::string::npos || k0 >= close) break;
            const size_t k1 = text.find('"', k0 + 1);
            const size_t colon = text.find(':', k1);
            if (k1 == std::string::npos || colon == std::string::npos || colon >= close) break;
            const std::string key = text.substr(k0 + 1, k1 - k0 - 1);
            size_t v = colon + 1;
            while (v < close && (text[v] == ' ' || text[v] == '\n' || text[v] == '\t')) ++v;
            std::string sval;
            double num = 0.0;
            if (v < close && text[v] == '"') {
                const size_t v1 = text.find('"', v + 1);
                sval = text.substr(v + 1, v1 - v - 1);
                p = v1 + 1;
            } else {
                char *endp = nullptr;
                num = std::strtod(text.c_str() + v, &endp);
                p = (size_t)(endp - text.c_str());
                if (p <= v) p = v + 1;
            }
            if (key == "arch") e.arch = sval;
            else if (key == "log2_t0") e.log2_t0 = (int)num;
            else if (key == "n_dur") e.n_dur = (int)num;
            else if (key == "log2_periods") e.log2_periods = (int)num;
            else if (key == "fold_period_block") e.tu.fold_period_block = (int)num;
            else if (key == "fold_wgs_per_cu") e.tu.fold_wgs_per_cu = (int)num;
            else if (key == "fold_units_per_wg") e.tu.fold_units_per_wg = (int)num;
            else if (key == "fold_variant") e.tu.fold_variant = (int)num;
            else if (key == "linear_windows") e.tu.linear_windows = (int)num;
            else if (key == "fold_ms") e.fold_ms = num;
            else if (key == "linear_ms") e.linear_ms = num;
            const size_t comma = text.find(',', p);
            p = (comma == std::string::npos || comma > close) ? close : comma + 1;
        }
        out.push_back(e);
        pos = close + 1;
    }
    return out;
}

// Writes every entry to a temporary file next to `path`, then renames it
// over `path` (a reader never sees a half-written cache).
int write_cache(const char *path, const std::vector<Entry> &entries) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) return set_error(CETRA_ERR_INVALID, "autotune: cannot write %s: %s", tmp.c_str(), std::strerror(errno));
    std::fprintf(fp, "{\n \"format\": \"cetra-autotune-1\",\n \"entries\": [\n");
    for (size_t i = 0; i < entries.size(); ++i) {
        const Entry &e = entries[i];
        std::fprintf(fp,
                     "  {\"arch\": \"%s\", \"log2_t0\": %d, \"n_dur\": %d, \"log2_periods\": %d, "
                     "\"fold_period_block\": %d, \"fold_wgs_per_cu\": %d, \"fold_units_per_wg\": %d, "
                     "\"fold_variant\": %d, \"linear_windows\": %d, \"fold_ms\": %.6g, \"linear_ms\": %.6g}%s\n",
                     e.arch.c_str(), e.log2_t0, e.n_dur, e.log2_periods, e.tu.fold_period_block,
                     e.tu.fold_wgs_per_cu, e.tu.fold_units_per_wg, e.tu.fold_variant, e.tu.linear_windows,
                     e.fold_ms, e.linear_ms, i + 1 < entries.size() ? "," : "");
    }
    std::fprintf(fp, " ]\n}\n");
    if (std::fclose(fp) != 0) return set_error(CETRA_ERR_INVALID, "autotune: cannot write %s", tmp.c_str());
    if (std::rename(tmp.c_str(), path) != 0)
        return set_error(CETRA_ERR_INVALID, "autotune: cannot replace %s: %s", path, std::strerror(errno));
    return CETRA_OK;
}

bool same_class(const Entry &e, const cetra_shape_class &s) {
    return e.arch == s.arch && e.log2_t0 == s.log2_t0 && e.n_dur == s.n_dur && e.log2_periods == s.log2_periods;
}

bool valid_tuning(const cetra_tuning &t) {
    cetra_tuning cur;
    if (cetra_get_tuning(&cur) != CETRA_OK) return false;
    const int rc = cetra_set_tuning(&t);  // validates; restores below
    cetra_set_tuning(&cur);
    return rc == CETRA_OK;
}

// Mean time of `reps` calls of fn after one untimed call, with HIP events on
// the stream.
template <class F>
int time_ms(hipStream_t s, int reps, F fn, double *ms) {
    int rc = fn();
    if (rc) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(CETRA_ERR_HIP, "autotune: hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(CETRA_ERR_HIP, "autotune: hipEventCreate");
    }
    hipError_t se = hipEventRecord(e0, s);
    for (int r = 0; r < reps && rc == CETRA_OK; ++r) rc = fn();
    if (se == hipSuccess) se = hipEventRecord(e1, s);
    if (se == hipSuccess) se = hipEventSynchronize(e1);
    float t = 0.0f;
    if (se == hipSuccess) se = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (se != hipSuccess) return set_error(CETRA_ERR_HIP, "autotune: %s", hipGetErrorString(se));
    *ms = (double)t / reps;
    return CETRA_OK;
}

}  // namespace

extern "C" int cetra_shape_class_of(const cetra_grid *grid, int64_t n_periods, cetra_shape_class *out) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(out && n_periods >= 1, "shape_class_of: NULL output or no periods");
    std::memset(out, 0, sizeof *out);
    out->log2_t0 = ceil_log2(grid->n_t0);
    out->n_dur = grid->n_dur;
    out->log2_periods = ceil_log2(n_periods);
    return CETRA_OK;
}

extern "C" int cetra_autotune_workspace(const cetra_grid *grid, int64_t n_periods, size_t *bytes) {
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(bytes && n_periods >= 1, "autotune_workspace: NULL output or no periods");
    const int64_t n = slice_periods(grid, n_periods);
    size_t fw = 0;
    if ((rc = cetra_periodic_workspace(grid, n, &fw))) return rc;
    *bytes = align256(fw) + 5 * align256(4 * (size_t)n);
    return CETRA_OK;
}

extern "C" int cetra_autotune(void *stream, const cetra_shape_class *shape, const cetra_grid *grid,
                              const float *flux, const float *ivar, const float *model, float *fold,
                              const double *periods, int64_t n_periods, void *work, size_t work_bytes,
                              const char *cache_path, cetra_tuning *out, double *fold_ms, double *linear_ms,
                              int32_t *from_cache) {
    clear_error();
    CETRA_REQUIRE(shape && out, "autotune: NULL shape or output");
    cetra_shape_class key = *shape;
    key.arch[sizeof key.arch - 1] = '\0';
    if (key.arch[0] == '\0') {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return set_error(CETRA_ERR_DEVICE, "autotune: no device to name the architecture");
        std::snprintf(key.arch, sizeof key.arch, "%s", prop.gcnArchName);
        char *colon = std::strchr(key.arch, ':');
        if (colon) *colon = '\0';
    }
    std::vector<Entry> entries = cache_path ? read_cache(cache_path) : std::vector<Entry>();
    for (const Entry &e : entries) {
        if (!same_class(e, key) || !valid_tuning(e.tu)) continue;
        int rc = cetra_set_tuning(&e.tu);
        if (rc) return rc;
        *out = e.tu;
        if (fold_ms) *fold_ms = e.fold_ms;
        if (linear_ms) *linear_ms = e.linear_ms;
        if (from_cache) *from_cache = 1;
        return CETRA_OK;
    }
    // not cached: time the candidates on the caller's data
    int rc = check_grid(grid);
    if (rc) return rc;
    CETRA_REQUIRE(flux && ivar && model && fold && periods && work, "autotune: NULL pointer");
    CETRA_REQUIRE(n_periods >= 1, "autotune: no periods");
    size_t need = 0;
    if ((rc = cetra_autotune_workspace(grid, n_periods, &need))) return rc;
    if (work_bytes < need) return set_error(CETRA_ERR_WORKSPACE, "autotune: workspace needs %zu bytes", need);
    hipStream_t s = as_stream(stream);
    cetra_tuning before;
    cetra_get_tuning(&before);
    cetra_tuning best = before;
    // linear search: windows per lane
    double best_lin = 1e300;
    for (int W : {1, 2, 4}) {
        cetra_tuning t = before;
        t.linear_windows = W;
        cetra_set_tuning(&t);
        double ms = 0.0;
        rc = time_ms(s, 2, [&] { return cetra_linear_search(stream, grid, flux, ivar, model, fold, nullptr, nullptr,
                                                            nullptr); }, &ms);
        if (rc) break;
        if (ms < best_lin) {
            best_lin = ms;
            best.linear_windows = W;
        }
    }
    // periodic search: launch shapes on a contiguous slice of the periods
    double best_fold = 1e300;
    if (rc == CETRA_OK) {
        const int64_t n = slice_periods(grid, n_periods);
        const double *p0 = periods + (n_periods - n) / 2;
        size_t fw = 0;
        cetra_periodic_workspace(grid, n, &fw);
        char *w = static_cast<char *>(work);
        float *o_lr = reinterpret_cast<float *>(w + align256(fw));
        int32_t *o_ep = reinterpret_cast<int32_t *>(w + align256(fw) + align256(4 * (size_t)n));
        int32_t *o_du = reinterpret_cast<int32_t *>(w + align256(fw) + 2 * align256(4 * (size_t)n));
        float *o_z = reinterpret_cast<float *>(w + align256(fw) + 3 * align256(4 * (size_t)n));
        float *o_zv = reinterpret_cast<float *>(w + align256(fw) + 4 * align256(4 * (size_t)n));
        std::vector<cetra_tuning> cands;
        for (int B : {4, 8, 16})
            for (int wg : {2, 4, 8})
                for (int u : {2, 4, 8})
                    for (int v : {0, 2}) {
                        cetra_tuning t = best;
                        t.fold_period_block = B;
                        t.fold_wgs_per_cu = wg;
                        t.fold_units_per_wg = u;
                        t.fold_variant = v;
                        cands.push_back(t);
                    }
        for (const cetra_tuning &t : cands) {
            cetra_set_tuning(&t);
            double ms = 0.0;
            rc = time_ms(s, 1, [&] {
                return cetra_periodic_search(stream, grid, fold, p0, n, nullptr, nullptr, 0, work, fw, o_lr, o_ep,
                                             o_du, o_z, o_zv);
            }, &ms);
            if (rc) break;
            if (ms < best_fold) {
                best_fold = ms;
                const int W = best.linear_windows;
                best = t;
                best.linear_windows = W;
            }
        }
    }
    if (rc) {
        cetra_set_tuning(&before);
        return rc;
    }
    if ((rc = cetra_set_tuning(&best))) return rc;
    *out = best;
    if (fold_ms) *fold_ms = best_fold;
    if (linear_ms) *linear_ms = best_lin;
    if (from_cache) *from_cache = 0;
    if (cache_path) {
        Entry e;
        e.arch = key.arch;
        e.log2_t0 = key.log2_t0;
        e.n_dur = key.n_dur;
        e.log2_periods = key.log2_periods;
        e.tu = best;
        e.fold_ms = best_fold;
        e.linear_ms = best_lin;
        entries.erase(std::remove_if(entries.begin(), entries.end(), [&](const Entry &x) { return same_class(x, key); }),
                      entries.end());
        entries.push_back(e);
        if ((rc = write_cache(cache_path, entries))) return rc;
    }
    return CETRA_OK;
}
