// Process-wide cache of tuned tilings, optionally persisted as JSON:
//   {"<key>": [tg_cap, passes, nper_cap, microseconds], ...}
#include "autotune.h"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

namespace sp {

namespace {

std::mutex g_mu;
std::map<std::string, TuneChoice> g_table;
bool g_loaded = false;

const char* cache_path() { return std::getenv("SEGPART_TUNE_CACHE"); }

// Minimal reader for the flat format written by save(): tolerant of
// whitespace, ignores anything it does not recognise.
void load() {
  g_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while (true) {
    size_t q0 = s.find('"', i);
    if (q0 == std::string::npos) break;
    size_t q1 = s.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    size_t b0 = s.find('[', q1);
    size_t b1 = s.find(']', b0 == std::string::npos ? q1 : b0);
    if (b0 == std::string::npos || b1 == std::string::npos) break;
    TuneChoice c;
    if (std::sscanf(s.substr(b0 + 1, b1 - b0 - 1).c_str(), "%d , %d , %d , %lf", &c.tg_cap,
                    &c.passes, &c.nper_cap, &c.us) == 4)
      g_table[s.substr(q0 + 1, q1 - q0 - 1)] = c;
    i = b1 + 1;
  }
}

void save() {
  const char* path = cache_path();
  if (!path) return;
  std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t k = 0;
    for (const auto& e : g_table) {
      f << "  \"" << e.first << "\": [" << e.second.tg_cap << ", " << e.second.passes << ", "
        << e.second.nper_cap << ", " << e.second.us << "]" << (++k < g_table.size() ? "," : "")
        << "\n";
    }
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

}  // namespace

bool tune_lookup(const std::string& key, TuneChoice* out) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_loaded) load();
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

void tune_store(const std::string& key, const TuneChoice& c) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_loaded) load();
  g_table[key] = c;
  save();
}

bool tune_enabled(bool dflt) {
  const char* e = std::getenv("SEGPART_AUTOTUNE");
  if (!e || !*e) return dflt;
  return std::atoi(e) != 0;
}

}  // namespace sp
