// Persistent cache of the autotuner's choices: a flat JSON object of string
// pairs ({"key": "value", ...}), read once per process and rewritten
// (temporary file, then rename) whenever a new choice is stored.  Keys carry
// the device architecture and a digest of the kernel sources, so a choice
// measured on other hardware or other kernels is never reused.
#include <dlfcn.h>
#include <unistd.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "mg_tune.h"

#ifndef MG_SOURCE_DIGEST
#define MG_SOURCE_DIGEST "unknown"
#endif

namespace mg {
namespace {

std::mutex g_mu;
bool g_loaded = false;
std::map<std::string, std::string> g_cache;

std::string find_cache_path() {
  const char* env = std::getenv("MG_TUNE_CACHE");
  if (env) return std::strcmp(env, "off") == 0 ? std::string() : std::string(env);
  Dl_info info{};
  if (dladdr(reinterpret_cast<void*>(&find_cache_path), &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t slash = p.rfind('/');
    return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/libmg_tune.json";
  }
  return std::string();
}

// The cache file, fixed at the first use in the process.
const std::string& cache_path() {
  static const std::string path = find_cache_path();
  return path;
}

// Reads the quoted strings of the file in order and pairs them up (keys and
// values never contain quotes or backslashes).
void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const std::string path = cache_path();
  if (path.empty()) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  std::string key;
  bool have_key = false;
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string tok = s.substr(i + 1, j - i - 1);
    if (have_key) {
      g_cache[key] = tok;
    } else {
      key = tok;
    }
    have_key = !have_key;
    i = j + 1;
  }
}

void save_locked() {
  const std::string path = cache_path();
  if (path.empty()) return;
  const std::string tmp = path + ".tmp" + std::to_string((long)::getpid());
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t k = 0;
    for (const auto& kv : g_cache) f << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++k < g_cache.size() ? ",\n" : "\n");
    f << "}\n";
    if (!f) return;
  }
  std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

std::string tune_identity() {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  return arch + "|" + MG_SOURCE_DIGEST;
}

std::string tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_locked();
  auto it = g_cache.find(key);
  return it == g_cache.end() ? std::string() : it->second;
}

void tune_store(const std::string& key, const std::string& value) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_locked();
  g_cache[key] = value;
  save_locked();
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

}  // namespace mg
