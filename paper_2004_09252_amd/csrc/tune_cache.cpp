// JSON cache of autotuned tilings.  One entry per line inside a JSON list so
// that the file is both valid JSON and trivially parsed here:
//   {"entries": [
//   {"arch": "gfx950:sramecc+:xnack-", "cus": 256, "bucket": 18, "ppw": 8,
//    "unroll": 1, "waves_per_cu": 32, "us": 512.25},
//   ...
//   ]}
#include "tune_cache.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace {

std::mutex g_mu;

struct Entry {
  std::string arch;
  int cus = 0;
  uint32_t bucket = 0, ppw = 0, unroll = 0, wpc = 0;
  double us = 0;
};

bool parse_line(const std::string& line, Entry* e) {
  const char* p = std::strstr(line.c_str(), "\"arch\": \"");
  if (!p) return false;
  p += 9;
  const char* q = std::strchr(p, '"');
  if (!q) return false;
  e->arch.assign(p, q - p);
  if (std::sscanf(q + 1,
                  ", \"cus\": %d, \"bucket\": %u, \"ppw\": %u, \"unroll\": %u, "
                  "\"waves_per_cu\": %u, \"us\": %lf",
                  &e->cus, &e->bucket, &e->ppw, &e->unroll, &e->wpc,
                  &e->us) != 6)
    return false;
  return e->ppw >= 1 && e->ppw <= 4096 && (e->unroll == 1 || e->unroll == 2) &&
         e->wpc >= 1 && e->wpc <= 256 && e->bucket < 64;
}

std::vector<Entry> read_all(const char* path) {
  std::vector<Entry> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    Entry e;
    if (parse_line(line, &e)) out.push_back(e);
  }
  return out;
}

}  // namespace

void ms_tune_cache_load(
    const char* arch, int cu_count,
    const std::function<void(uint32_t, uint32_t, uint32_t, uint32_t, double)>&
        fn) {
  const char* path = std::getenv("MS_TUNE_CACHE");
  if (!path || !*path) return;
  std::lock_guard<std::mutex> lk(g_mu);
  for (const Entry& e : read_all(path))
    if (e.arch == arch && e.cus == cu_count)
      fn(e.bucket, e.ppw, e.unroll, e.wpc, e.us);
}

void ms_tune_cache_store(const char* arch, int cu_count, uint32_t bucket,
                         uint32_t ppw, uint32_t unroll, uint32_t waves_per_cu,
                         double us) {
  const char* path = std::getenv("MS_TUNE_CACHE");
  if (!path || !*path) return;
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<Entry> all = read_all(path);
  bool replaced = false;
  for (Entry& e : all)
    if (e.arch == arch && e.cus == cu_count && e.bucket == bucket) {
      e.ppw = ppw;
      e.unroll = unroll;
      e.wpc = waves_per_cu;
      e.us = us;
      replaced = true;
    }
  if (!replaced) {
    Entry e;
    e.arch = arch;
    e.cus = cu_count;
    e.bucket = bucket;
    e.ppw = ppw;
    e.unroll = unroll;
    e.wpc = waves_per_cu;
    e.us = us;
    all.push_back(e);
  }
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    f << "{\"entries\": [\n";
    for (size_t i = 0; i < all.size(); ++i) {
      char buf[512];
      std::snprintf(buf, sizeof(buf),
                    "{\"arch\": \"%s\", \"cus\": %d, \"bucket\": %u, \"ppw\": "
                    "%u, \"unroll\": %u, \"waves_per_cu\": %u, \"us\": %.3f}%s\n",
                    all[i].arch.c_str(), all[i].cus, all[i].bucket,
                    all[i].ppw, all[i].unroll, all[i].wpc, all[i].us,
                    i + 1 < all.size() ? "," : "");
      f << buf;
    }
    f << "]}\n";
  }
  std::rename(tmp.c_str(), path);
}
