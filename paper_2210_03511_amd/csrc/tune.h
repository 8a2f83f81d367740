// Autotuning helpers: a fingerprint of what a choice was tuned for, and a
// plain-text cache file of choices (one line per choice:
// "symed-tune 1 <kind> <fingerprint> <mode> <a> <b> <seconds>").
#pragma once

#include <cstdint>
#include <string>

namespace symed {

// FNV-1a over a byte range, continuing from h.
uint64_t fnv1a(const void *data, size_t n, uint64_t h = 0xcbf29ce484222325ull);
// Device identity for fingerprints: name and compute-unit count.
uint64_t device_fingerprint(int device);
// Look up a choice (a, b) of `kind` for (fp, mode); false if absent or unreadable.
bool tune_cache_lookup(const char *path, const char *kind, uint64_t fp, int mode, int64_t &a, int64_t &b);
// Append a choice; false if the file cannot be written.
bool tune_cache_store(const char *path, const char *kind, uint64_t fp, int mode, int64_t a, int64_t b, double seconds);

}  // namespace symed
