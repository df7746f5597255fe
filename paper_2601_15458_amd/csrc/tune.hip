// Tuning table: per (kind, alphabet size, length bin) the launch variant the
// library uses instead of its default, filled by the autotune entry points
// (lev.hip, nw.hip) or imported from a JSON cache.  Host code only.
//
// Kinds and values:
//   MSA_TUNE_LEV (0): bin = pattern words ceil(max_len / 64) of the set A;
//                     value = words per pass of the kernel variant.
//   MSA_TUNE_NW  (1): bin = wavefronts per pair ceil(ceil(max_len_A / 32) / 64);
//                     value = steps between workgroup barriers of the fill.
//   MSA_TUNE_PAIRS (3): bin = pattern words of the longer set of a pair list;
//                     value = layout: 1 (a pair per lane), 2 (a pair per
//                     group of lanes) or 64 (64 pairs share a pattern).
//   MSA_TUNE_TREE (2): bin = pattern words ceil(max_len / 64) of the set;
//                     value = words per pass of the tree build's kernels.
//   MSA_TUNE_TREE_XL (4): bin as for MSA_TUNE_TREE; value = words per lane
//                     and cluster-size caps of the across-lanes passes.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "common.hpp"
#include "lev_core.hpp"
#include "lev_xl.hpp"

namespace msadp {

namespace {
std::mutex g_mu;
std::map<std::tuple<int, int, int>, int> g_table;

bool valid_value(int kind, int value) {
    if (kind == MSA_TUNE_LEV) return is_lev_class(value);
    if (kind == MSA_TUNE_NW) return value == 16 || value == 32 || value == 64;
    if (kind == MSA_TUNE_TREE) return is_tree_class(value);
    if (kind == MSA_TUNE_PAIRS) return value == 1 || value == 2 || value == kWave;
    if (kind == MSA_TUNE_TREE_XL) return xl_value_valid(value);
    return false;
}

bool valid_key(int kind, int sigma, int bin) {
    return (kind == MSA_TUNE_LEV || kind == MSA_TUNE_NW || kind == MSA_TUNE_TREE ||
            kind == MSA_TUNE_PAIRS || kind == MSA_TUNE_TREE_XL) &&
           sigma >= 2 && sigma <= 33 &&
           bin >= 1 && bin <= (1 << 20);
}

// gfx name of the current device without feature suffixes ("gfx950").
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
        return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}
}  // namespace

int tuned_value(int kind, int sigma, int bin, int fallback) {
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_table.find({kind, sigma, bin});
    return it == g_table.end() ? fallback : it->second;
}

}  // namespace msadp

using namespace msadp;

extern "C" {

int msa_tune_set(int32_t kind, int32_t sigma, int32_t bin, int32_t value) {
    if (!valid_key(kind, sigma, bin) || !valid_value(kind, value)) return MSA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[{kind, sigma, bin}] = value;
    return MSA_OK;
}

int msa_tune_get(int32_t kind, int32_t sigma, int32_t bin, int32_t *value) {
    if (value == nullptr || !valid_key(kind, sigma, bin)) return MSA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_table.find({kind, sigma, bin});
    *value = it == g_table.end() ? 0 : it->second;
    return MSA_OK;
}

int msa_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    return MSA_OK;
}

int msa_tune_candidates(int32_t kind, int32_t *values, int32_t cap, int32_t *count) {
    if (count == nullptr || cap < 0 || (cap > 0 && values == nullptr)) return MSA_EINVAL;
    int n = 0;
    if (kind == MSA_TUNE_LEV) {
        for (int c : kLevClasses) {
            if (n < cap) values[n] = c;
            ++n;
        }
    } else if (kind == MSA_TUNE_TREE) {
        for (int c : kTreeClasses) {
            if (n < cap) values[n] = c;
            ++n;
        }
    } else if (kind == MSA_TUNE_NW) {
        for (int r : {16, 32, 64}) {
            if (n < cap) values[n] = r;
            ++n;
        }
    } else if (kind == MSA_TUNE_PAIRS) {
        for (int r : {1, 2, kWave}) {
            if (n < cap) values[n] = r;
            ++n;
        }
    } else if (kind == MSA_TUNE_TREE_XL) {
        for (const int v : kXlCandidates) {
            if (n < cap) values[n] = v;
            ++n;
        }
    } else {
        return MSA_EINVAL;
    }
    *count = n;
    return n <= cap ? MSA_OK : MSA_ENOSPC;
}

int msa_tune_export(char *buf, size_t cap, size_t *len) {
    if (len == nullptr || (cap > 0 && buf == nullptr)) return MSA_EINVAL;
    std::string out = "{\"arch\": \"" + device_arch() + "\", \"entries\": [";
    {
        std::lock_guard<std::mutex> lk(g_mu);
        bool first = true;
        for (const auto &e : g_table) {
            char item[96];
            std::snprintf(item, sizeof(item), "%s[%d, %d, %d, %d]", first ? "" : ", ",
                          std::get<0>(e.first), std::get<1>(e.first), std::get<2>(e.first),
                          e.second);
            out += item;
            first = false;
        }
    }
    out += "]}";
    *len = out.size();
    if (out.size() + 1 > cap) return MSA_ENOSPC;
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return MSA_OK;
}

int msa_tune_import(const char *json) {
    if (json == nullptr) return MSA_EINVAL;
    const std::string s(json);
    // "arch": "<name>" must name this device
    const size_t ak = s.find("\"arch\"");
    if (ak == std::string::npos) return MSA_EINVAL;
    const size_t q0 = s.find('"', s.find(':', ak) + 1);
    const size_t q1 = q0 == std::string::npos ? q0 : s.find('"', q0 + 1);
    if (q1 == std::string::npos) return MSA_EINVAL;
    if (s.substr(q0 + 1, q1 - q0 - 1) != device_arch()) return MSA_EINVAL;
    const size_t ek = s.find("\"entries\"");
    if (ek == std::string::npos) return MSA_EINVAL;
    size_t pos = s.find('[', ek);
    if (pos == std::string::npos) return MSA_EINVAL;
    std::map<std::tuple<int, int, int>, int> parsed;
    ++pos;
    for (;;) {
        const size_t open = s.find('[', pos), close_all = s.find(']', pos);
        if (open == std::string::npos || close_all < open) break;   // end of the list
        int k, sg, b, v;
        if (std::sscanf(s.c_str() + open, "[%d , %d , %d , %d ]", &k, &sg, &b, &v) != 4)
            return MSA_EINVAL;
        if (!valid_key(k, sg, b) || !valid_value(k, v)) return MSA_EINVAL;
        parsed[{k, sg, b}] = v;
        pos = s.find(']', open);
        if (pos == std::string::npos) return MSA_EINVAL;
        ++pos;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &e : parsed) g_table[e.first] = e.second;
    return MSA_OK;
}

}  // extern "C"
