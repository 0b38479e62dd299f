// tune_cache.hip - the batch autotuner's cache of launch shapes (host code).
//
// A shape is chosen by timing every candidate once per problem signature
// (batch.hip).  The result is kept in memory and in a JSON file, so that
// later processes on the same kind of device reuse it instead of timing
// again.  The key is the device's architecture name, its compute-unit count
// and the batch signature (every job's size, depth, sphere and light count
// and skybox flag); the file stores a 64-bit FNV-1a digest of the key with
// its length.
//
// File: $RT_TUNE_CACHE if set (an empty value keeps the cache in memory only),
// else $XDG_CACHE_HOME/rtmi/tune.json, else $HOME/.cache/rtmi/tune.json.
// Format, one entry per line:
//   {"format": "rtmi-tune-cache-1", "entries": {
//    "<digest>": {"workgroups": 2048, "wave_w": 16, "waves": 4},
//    ...
//   }}
// Reading tolerates anything else: a line that does not parse, or a shape
// outside the candidates the tuner times, is ignored.  Writing re-reads the
// file, adds the entry and replaces the file by rename, so a reader never
// sees a half-written file; two processes storing at once may lose one of
// the two entries, never the file.
#include <errno.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <map>
#include <mutex>
#include <string>

#include "rt_internal.hpp"

namespace rtk {

namespace {

std::mutex g_mu;
std::map<std::string, TunedShape> g_mem;   // full key -> shape

const char* kFormat = "rtmi-tune-cache-1";

std::string digest(const std::string& key) {
  uint64_t h = 1469598103934665603ull;   // FNV-1a 64-bit offset basis
  for (unsigned char ch : key) {
    h ^= ch;
    h *= 1099511628211ull;                // FNV 64-bit prime
  }
  char buf[48];
  snprintf(buf, sizeof buf, "%016llx:%zu", (unsigned long long)h, key.size());
  return buf;
}

std::string cache_path() {
  const char* env = getenv("RT_TUNE_CACHE");
  if (env) return env;   // empty: memory only
  const char* xdg = getenv("XDG_CACHE_HOME");
  if (xdg && *xdg) return std::string(xdg) + "/rtmi/tune.json";
  const char* home = getenv("HOME");
  if (home && *home) return std::string(home) + "/.cache/rtmi/tune.json";
  return "";
}

// Creates the directories above `path` (mode 0755); true if they exist after.
bool make_parent_dirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i) {
    if (path[i] != '/') continue;
    const std::string dir = path.substr(0, i);
    if (mkdir(dir.c_str(), 0755) != 0 && errno != EEXIST) return false;
  }
  return true;
}

// Entries of the file at `path` (digest -> shape); empty if it is missing or
// not in the format.
std::map<std::string, TunedShape> read_file(const std::string& path) {
  std::map<std::string, TunedShape> out;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return out;
  char line[512];
  bool format_ok = false;
  while (fgets(line, sizeof line, f)) {
    if (!format_ok) {
      format_ok = strstr(line, kFormat) != nullptr;
      continue;
    }
    char key[64];
    TunedShape s;
    if (sscanf(line, " \"%47[0-9a-f:]\": {\"workgroups\": %d, \"wave_w\": %d, \"waves\": %d",
               key, &s.grid, &s.wave_w, &s.waves) == 4 &&
        tuned_shape_valid(s))
      out[key] = s;
  }
  fclose(f);
  return out;
}

bool write_file(const std::string& path, const std::map<std::string, TunedShape>& entries) {
  if (!make_parent_dirs(path)) return false;
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\"format\": \"%s\", \"entries\": {\n", kFormat);
  size_t i = 0;
  for (const auto& kv : entries) {
    fprintf(f, " \"%s\": {\"workgroups\": %d, \"wave_w\": %d, \"waves\": %d}%s\n",
            kv.first.c_str(), kv.second.grid, kv.second.wave_w, kv.second.waves,
            ++i < entries.size() ? "," : "");
  }
  fprintf(f, "}}\n");
  const bool ok = fflush(f) == 0 && fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), path.c_str()) != 0) {
    unlink(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace

bool tuned_shape_valid(const TunedShape& s) {
  const bool ww = s.wave_w == 8 || s.wave_w == 16 || s.wave_w == 64;
  const bool wv = s.waves == 1 || s.waves == 2 || s.waves == 4;
  return ww && wv && s.grid >= 1 && s.grid <= (1 << 20);
}

bool tune_cache_get(const std::string& key, TunedShape* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_mem.find(key);
  if (it != g_mem.end()) {
    *out = it->second;
    return true;
  }
  const std::string path = cache_path();
  if (path.empty()) return false;
  const auto entries = read_file(path);
  auto jt = entries.find(digest(key));
  if (jt == entries.end()) return false;
  g_mem[key] = jt->second;
  *out = jt->second;
  return true;
}

bool tune_cache_put(const std::string& key, const TunedShape& s) {
  if (!tuned_shape_valid(s)) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  g_mem[key] = s;
  const std::string path = cache_path();
  if (path.empty()) return true;
  auto entries = read_file(path);
  entries[digest(key)] = s;
  return write_file(path, entries);
}

void tune_cache_forget_memory() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_mem.clear();
}

}  // namespace rtk

using namespace rtk;

extern "C" {

rt_status rt_tune_cache_get(const char* key, int32_t* workgroups, int32_t* tile_w,
                            int32_t* tile_h, int32_t* found) {
  if (!key || !found) return fail(RT_ERR_INVALID_ARG, "key or found is NULL");
  TunedShape s;
  *found = tune_cache_get(key, &s) ? 1 : 0;
  if (*found) {
    if (workgroups) *workgroups = s.grid;
    if (tile_w) *tile_w = s.wave_w;
    if (tile_h) *tile_h = (64 / s.wave_w) * s.waves;
  }
  return RT_OK;
}

rt_status rt_tune_cache_put(const char* key, int32_t workgroups, int32_t tile_w,
                            int32_t tile_h) {
  if (!key) return fail(RT_ERR_INVALID_ARG, "key is NULL");
  TunedShape s;
  s.grid = workgroups;
  s.wave_w = tile_w;
  s.waves = (tile_w > 0 && tile_w <= 64 && tile_h > 0 && tile_h <= 256 && (tile_w * tile_h) % 64 == 0)
                ? tile_w * tile_h / 64
                : 0;
  if (!tuned_shape_valid(s) || (64 / s.wave_w) * s.waves != tile_h)
    return fail(RT_ERR_INVALID_ARG,
                "shape %d workgroups of %dx%d tiles is not one the tuner picks from", workgroups,
                tile_w, tile_h);
  if (!tune_cache_put(key, s))
    return fail(RT_ERR_UNSUPPORTED, "could not write the tune cache file %s",
                cache_path().c_str());
  return RT_OK;
}

rt_status rt_tune_cache_forget(void) {
  tune_cache_forget_memory();
  return RT_OK;
}

}  // extern "C"
