// tune_cache.h -- the autotuner's result cache (tune_cache.cpp).
#pragma once

#include <string>

#include "aesgpu.h"

namespace aesgpu {

// Signature of a batch for the cache: device architecture and compute units,
// and size classes (floor of log2) of the request count, of the requests per
// op, of the total payload, of the shortest and longest non-empty request and
// of the number of schedules.
std::string tune_signature(const char *arch, int n_cu, const aes_req_t *reqs, uint64_t n,
                           uint32_t n_scheds);

// The configuration stored for sig in the cache file at path (the last entry
// of that signature); false if the file or the entry is missing.
bool tune_cache_lookup(const char *path, const std::string &sig, aes_launch_config_t *out);

// Stores c for sig, replacing that signature's entries; false on an I/O error.
bool tune_cache_store(const char *path, const std::string &sig, const aes_launch_config_t &c);

}  // namespace aesgpu
