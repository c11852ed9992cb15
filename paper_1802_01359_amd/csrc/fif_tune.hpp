// Plan choices of one signal length (what the autotuner picks) and their
// on-disk cache.  Host code only.
//
// Cache file: one entry per line,
//   FIFTUNE1 <device key> <N> <N1> <N2> <TC> <TR> <radices 1> <radices 2> <us> <us_default>
// radices written as d.d.d (first pass first, "-" for none), the device key
// without white space.  Lines that do not parse, or whose choice is not a
// valid plan of their length, are ignored; a store rewrites the file through
// a temporary file and a rename, keeping every other valid line.
#pragma once
#include <stdint.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include "../../include/fif.h"
#include "fif_types.hpp"

namespace fif {

inline bool radix_ok(int r) { return r == 2 || r == 3 || r == 4 || r == 5 || r == 7 || r == 8; }

// Product of a radix list, or -1 if a radix is not one the kernels have.
inline int64_t radix_product(const int8_t* rad, int n)
{
    if (n < 0 || n > kMaxRadices) return -1;
    int64_t p = 1;
    for (int i = 0; i < n; ++i) {
        if (!radix_ok(rad[i])) return -1;
        p *= rad[i];
    }
    return p;
}

// A choice is a valid plan of length N: one LDS pass (N <= kFftCap, N1 = 1,
// N2 = N, TC = TR = 1, radices of N) or a four-step split N = N1 * N2 with
// both factors <= kTileCap, tiles that divide their dimension and fit
// kTileCapBig elements, and radices of N2 (first list) and N1 (second).
inline bool choice_valid(const fif_length_plan& c)
{
    const int64_t N = c.N;
    if (N < 2) return false;
    if (N <= kFftCap) {
        return c.N1 == 1 && c.N2 == N && c.TC == 1 && c.TR == 1 && c.n_rad2 == 0 &&
               radix_product(c.rad1, c.n_rad1) == N;
    }
    if (c.N1 < 2 || c.N2 < 2 || c.N1 > kTileCap || c.N2 > kTileCap || (int64_t)c.N1 * c.N2 != N) return false;
    if (c.TC < 1 || c.N1 % c.TC || (int64_t)c.TC * c.N2 > kTileCapBig) return false;
    if (c.TR < 1 || c.N2 % c.TR || (int64_t)c.TR * c.N1 > kTileCapBig) return false;
    return radix_product(c.rad1, c.n_rad1) == c.N2 && radix_product(c.rad2, c.n_rad2) == c.N1;
}

inline std::string radix_text(const int8_t* rad, int n)
{
    if (n == 0) return "-";
    std::string s;
    for (int i = 0; i < n; ++i) {
        if (i) s += ".";
        s += std::to_string((int)rad[i]);
    }
    return s;
}

inline bool radix_parse(const std::string& t, int8_t* rad, int32_t& n)
{
    n = 0;
    if (t == "-") return true;
    std::stringstream ss(t);
    std::string part;
    while (std::getline(ss, part, '.')) {
        if (part.empty() || part.size() > 2 || n >= kMaxRadices) return false;
        for (char ch : part)
            if (ch < '0' || ch > '9') return false;
        rad[n++] = (int8_t)std::atoi(part.c_str());
    }
    return n > 0;
}

inline std::string key_text(const char* key)
{
    std::string k = key ? key : "";
    for (char& ch : k)
        if (ch == ' ' || ch == '\t' || ch == '\n' || ch == '\r') ch = '_';
    return k.empty() ? std::string("-") : k;
}

// Parse one cache line; false if it is not a valid entry.
inline bool parse_entry(const std::string& line, std::string& key, fif_length_plan& c)
{
    std::istringstream is(line);
    std::string tag, r1, r2;
    long long N = 0;
    int N1 = 0, N2 = 0, TC = 0, TR = 0;
    double us = 0.0, us0 = 0.0;
    if (!(is >> tag >> key >> N >> N1 >> N2 >> TC >> TR >> r1 >> r2 >> us >> us0)) return false;
    std::string rest;
    if (is >> rest) return false;
    if (tag != "FIFTUNE1") return false;
    std::memset(&c, 0, sizeof(c));
    c.N = N;
    c.N1 = N1;
    c.N2 = N2;
    c.TC = TC;
    c.TR = TR;
    c.us = us;
    c.us_default = us0;
    if (!radix_parse(r1, c.rad1, c.n_rad1) || !radix_parse(r2, c.rad2, c.n_rad2)) return false;
    return choice_valid(c);
}

inline std::string format_entry(const std::string& key, const fif_length_plan& c)
{
    char buf[128];
    std::snprintf(buf, sizeof(buf), " %lld %d %d %d %d ", (long long)c.N, c.N1, c.N2, c.TC, c.TR);
    char tail[64];
    std::snprintf(tail, sizeof(tail), " %.3f %.3f", c.us, c.us_default);
    return "FIFTUNE1 " + key + buf + radix_text(c.rad1, c.n_rad1) + " " + radix_text(c.rad2, c.n_rad2) + tail;
}

inline std::vector<std::string> read_lines(const char* path)
{
    std::vector<std::string> out;
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line)) out.push_back(line);
    return out;
}

// Last valid entry for (key, N); FIF_ERR_NOT_FOUND if none.
inline fif_status cache_lookup(const char* path, const char* key_in, int64_t N, fif_length_plan* out)
{
    if (!path || !out) return FIF_ERR_INVALID_ARG;
    const std::string want = key_text(key_in);
    bool found = false;
    for (const auto& line : read_lines(path)) {
        std::string key;
        fif_length_plan c;
        if (parse_entry(line, key, c) && key == want && c.N == N) {
            *out = c;
            found = true;
        }
    }
    return found ? FIF_OK : FIF_ERR_NOT_FOUND;
}

// Store c under key: valid lines for other (key, N) are kept, others dropped.
inline fif_status cache_store(const char* path, const char* key_in, const fif_length_plan& c)
{
    if (!path) return FIF_ERR_INVALID_ARG;
    if (!choice_valid(c)) return FIF_ERR_INVALID_ARG;
    const std::string key = key_text(key_in);
    std::vector<std::string> keep;
    for (const auto& line : read_lines(path)) {
        std::string k;
        fif_length_plan e;
        if (parse_entry(line, k, e) && !(k == key && e.N == c.N)) keep.push_back(line);
    }
    keep.push_back(format_entry(key, c));
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return FIF_ERR_INVALID_ARG;
        for (const auto& l : keep) f << l << "\n";
        if (!f) return FIF_ERR_INVALID_ARG;
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return FIF_ERR_INVALID_ARG;
    }
    return FIF_OK;
}

}  // namespace fif
