// Autotuning cache file (see tune_cache.h): a small line-oriented reader and
// writer for the one JSON layout the library itself writes,
//   {
//   "key": {"field": 1, "other": 2},
//   ...
//   }
// Lines that do not parse are skipped, so a damaged file costs a re-tune.
#include "tune_cache.h"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <unistd.h>

namespace mx {

namespace {

std::mutex g_cache_mu;

const char* cache_path() {
  const char* p = std::getenv("MX_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

bool parse_line(const std::string& line, std::string& key, TuneFields& f) {
  const size_t a = line.find('"');
  if (a == std::string::npos) return false;
  const size_t b = line.find('"', a + 1);
  if (b == std::string::npos) return false;
  const size_t o = line.find('{', b);
  const size_t e = o == std::string::npos ? o : line.find('}', o);
  if (e == std::string::npos) return false;
  key = line.substr(a + 1, b - a - 1);
  f.clear();
  size_t p = o + 1;
  for (;;) {
    const size_t q1 = line.find('"', p);
    if (q1 == std::string::npos || q1 > e) break;
    const size_t q2 = line.find('"', q1 + 1);
    if (q2 == std::string::npos || q2 > e) return false;
    const size_t c = line.find(':', q2);
    if (c == std::string::npos || c > e) return false;
    const char* s = line.c_str() + c + 1;
    char* end = nullptr;
    const long long v = std::strtoll(s, &end, 10);
    if (end == s) return false;
    f[line.substr(q1 + 1, q2 - q1 - 1)] = v;
    p = (size_t)(end - line.c_str());
  }
  return !key.empty();
}

std::map<std::string, TuneFields> load(const char* path) {
  std::map<std::string, TuneFields> m;
  std::ifstream in(path);
  std::string line, key;
  TuneFields f;
  while (std::getline(in, line))
    if (parse_line(line, key, f)) m[key] = f;
  return m;
}

}  // namespace

bool tune_cache_get(const std::string& key, TuneFields& out) {
  const char* path = cache_path();
  if (!path) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  const auto m = load(path);
  const auto it = m.find(key);
  if (it == m.end()) return false;
  out = it->second;
  return true;
}

void tune_cache_put(const std::string& key, const TuneFields& fields) {
  const char* path = cache_path();
  if (!path) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto m = load(path);
  m[key] = fields;
  std::ostringstream os;
  os << "{\n";
  size_t n = 0;
  for (const auto& kv : m) {
    os << "\"" << kv.first << "\": {";
    size_t i = 0;
    for (const auto& fv : kv.second) os << (i++ ? ", " : "") << "\"" << fv.first << "\": " << fv.second;
    os << "}" << (++n < m.size() ? "," : "") << "\n";
  }
  os << "}\n";
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return;
    out << os.str();
    if (!out.good()) {
      out.close();
      std::remove(tmp.c_str());
      return;
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}

}  // namespace mx
