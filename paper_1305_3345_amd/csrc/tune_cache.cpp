// tune_cache.cpp -- the autotuner's result cache: a text file that maps a
// batch's signature (device, request counts per op, size classes) to the
// launch configuration the tuner chose for it, so that a later process tuning
// a batch of the same shape applies the stored configuration instead of
// timing candidates again.
//
// File format, one entry per line (lines starting with '#' are comments):
//   <signature> TAB <12 unsigned integers: the aes_launch_config_t fields
//   tile_bytes .. chain_quad in declaration order>
// Lines that do not parse are skipped.  Writes replace the entry of the same
// signature, keep the others, and go through a temporary file renamed over
// the cache, so a reader never sees a half-written file.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <atomic>
#include <string>
#include <vector>

#include "tune_cache.h"

namespace aesgpu {

namespace {

// floor(log2(x)) as "2^k", or "-" for 0.
std::string size_class(uint64_t x) {
    if (!x)
        return "-";
    int k = 63 - __builtin_clzll(x);
    return "2^" + std::to_string(k);
}

constexpr int N_FIELDS = 12;

void config_fields(const aes_launch_config_t &c, uint32_t f[N_FIELDS]) {
    const uint32_t v[N_FIELDS] = {c.tile_bytes, c.ctr_nb,   c.ctr_wg, c.dec_nb,
                                  c.dec_wg,     c.chain_lanes, c.chain_wg, c.mixed_nb,
                                  c.fuse,       c.grid,     c.ctr_variant, c.chain_quad};
    memcpy(f, v, sizeof(v));
}

aes_launch_config_t config_of(const uint32_t f[N_FIELDS]) {
    aes_launch_config_t c;
    memset(&c, 0, sizeof(c));
    c.tile_bytes = f[0];
    c.ctr_nb = f[1];
    c.ctr_wg = f[2];
    c.dec_nb = f[3];
    c.dec_wg = f[4];
    c.chain_lanes = f[5];
    c.chain_wg = f[6];
    c.mixed_nb = f[7];
    c.fuse = f[8];
    c.grid = f[9];
    c.ctr_variant = f[10];
    c.chain_quad = f[11];
    return c;
}

// Splits "signature\tfields" and parses the fields; false for a line that
// is not an entry.
bool parse_entry(const std::string &line, std::string *sig, uint32_t f[N_FIELDS]) {
    const size_t tab = line.find('\t');
    if (line.empty() || line[0] == '#' || tab == std::string::npos || tab == 0)
        return false;
    *sig = line.substr(0, tab);
    const char *p = line.c_str() + tab + 1;
    for (int i = 0; i < N_FIELDS; i++) {
        char *end = nullptr;
        const unsigned long v = strtoul(p, &end, 10);
        if (end == p || v > 0xFFFFFFFFul)
            return false;
        f[i] = (uint32_t)v;
        p = end;
    }
    while (*p == ' ' || *p == '\t' || *p == '\r')
        p++;
    return *p == '\0';
}

bool read_lines(const char *path, std::vector<std::string> *lines) {
    FILE *fp = fopen(path, "r");
    if (!fp)
        return false;
    std::string cur;
    int ch;
    while ((ch = fgetc(fp)) != EOF) {
        if (ch == '\n') {
            lines->push_back(cur);
            cur.clear();
        } else {
            cur.push_back((char)ch);
        }
    }
    if (!cur.empty())
        lines->push_back(cur);
    fclose(fp);
    return true;
}

}  // namespace

std::string tune_signature(const char *arch, int n_cu, const aes_req_t *reqs, uint64_t n,
                           uint32_t n_scheds) {
    uint64_t per_op[5] = {0, 0, 0, 0, 0};
    uint64_t bytes = 0, min_len = 0, max_len = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (reqs[i].op < 5)
            per_op[reqs[i].op]++;
        const uint64_t len = reqs[i].length;
        if (!len)
            continue;
        bytes += len;
        min_len = (min_len == 0 || len < min_len) ? len : min_len;
        max_len = len > max_len ? len : max_len;
    }
    std::string s = "arch=" + std::string(arch ? arch : "?") + " cu=" + std::to_string(n_cu) +
                    " n=" + size_class(n) + " ops=";
    for (int op = 0; op < 5; op++)
        s += (op ? "," : "") + size_class(per_op[op]);
    s += " bytes=" + size_class(bytes) + " len=" + size_class(min_len) + ".." +
         size_class(max_len) + " keys=" + size_class(n_scheds);
    return s;
}

bool tune_cache_lookup(const char *path, const std::string &sig, aes_launch_config_t *out) {
    std::vector<std::string> lines;
    if (!path || !read_lines(path, &lines))
        return false;
    bool found = false;
    for (const std::string &ln : lines) {
        std::string s;
        uint32_t f[N_FIELDS];
        if (parse_entry(ln, &s, f) && s == sig) {
            *out = config_of(f);  // the last entry of a signature wins
            found = true;
        }
    }
    return found;
}

bool tune_cache_store(const char *path, const std::string &sig, const aes_launch_config_t &c) {
    if (!path || sig.find('\t') != std::string::npos || sig.find('\n') != std::string::npos)
        return false;
    std::vector<std::string> lines, keep;
    read_lines(path, &lines);  // a missing file starts empty
    for (const std::string &ln : lines) {
        std::string s;
        uint32_t f[N_FIELDS];
        if (!parse_entry(ln, &s, f) || s != sig)
            keep.push_back(ln);
    }
    uint32_t f[N_FIELDS];
    config_fields(c, f);
    std::string entry = sig + "\t";
    for (int i = 0; i < N_FIELDS; i++)
        entry += (i ? " " : "") + std::to_string(f[i]);
    keep.push_back(entry);
    // Unique per process and call: two threads (each with its own context)
    // may store at the same time; each renames only its own complete file.
    static std::atomic<uint64_t> seq{0};
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid()) + "." +
                            std::to_string(seq.fetch_add(1, std::memory_order_relaxed));
    FILE *fp = fopen(tmp.c_str(), "w");
    if (!fp)
        return false;
    bool ok = true;
    for (const std::string &ln : keep)
        ok = ok && fputs(ln.c_str(), fp) >= 0 && fputc('\n', fp) != EOF;
    ok = (fclose(fp) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        (void)remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace aesgpu
