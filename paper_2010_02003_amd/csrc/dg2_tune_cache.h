// Host-side cache of tuned launch shapes: a small JSON file mapping a key
// (GPU architecture, precision, variant, flux, kernel form and size class)
// to the launch shape the autotuner chose for it, so that a later context or
// batch with the same key takes the shape without timing candidates again.
//
// File format (written by this code, one entry per line):
//   {
//    "gfx950|fp32|NL|HLL|fused|4096x4096": {"rows": 48, "waves": 4, "graph_steps": 0, "ms": 0.4512},
//    ...
//   }
// Readers accept exactly this layout; a file that does not parse is treated
// as empty and rewritten.  Writers replace the whole file (write to a
// temporary name, then rename), so a reader never sees half a file;
// concurrent writers may drop each other's new entries.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

namespace dg2 {

struct TuneEntry {
  int rows = 0, waves = 4, graph_steps = 0;
  double ms = 0.0;
};

// Architecture name of the current device ("gfx950"), or "unknown".
inline std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

// Size class of an extent: the next power of two.
inline long long size_class(long long n) {
  long long c = 1;
  while (c < n) c <<= 1;
  return c;
}

inline bool parse_int_field(const std::string &line, const char *name, int &out) {
  const std::string key = std::string("\"") + name + "\":";
  const size_t p = line.find(key);
  if (p == std::string::npos) return false;
  return std::sscanf(line.c_str() + p + key.size(), " %d", &out) == 1;
}

inline std::map<std::string, TuneEntry> read_tune_cache(const std::string &path) {
  std::map<std::string, TuneEntry> m;
  std::ifstream f(path);
  if (!f) return m;
  std::string line;
  while (std::getline(f, line)) {
    const size_t q0 = line.find('"');
    const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
    if (q1 == std::string::npos || line.find("\": {", q1) != q1) continue;
    TuneEntry e;
    if (!parse_int_field(line, "rows", e.rows) || !parse_int_field(line, "waves", e.waves) ||
        !parse_int_field(line, "graph_steps", e.graph_steps))
      continue;
    const size_t pm = line.find("\"ms\":");
    if (pm != std::string::npos) std::sscanf(line.c_str() + pm + 5, " %lf", &e.ms);
    m[line.substr(q0 + 1, q1 - q0 - 1)] = e;
  }
  return m;
}

// Add or replace one entry; returns false if the file cannot be written.
inline bool write_tune_cache(const std::string &path, const std::string &key, const TuneEntry &e) {
  std::map<std::string, TuneEntry> m = read_tune_cache(path);
  m[key] = e;
  std::ostringstream s;
  s << "{\n";
  size_t k = 0;
  for (const auto &kv : m) {
    char buf[160];
    std::snprintf(buf, sizeof(buf), "{\"rows\": %d, \"waves\": %d, \"graph_steps\": %d, \"ms\": %.6g}",
                  kv.second.rows, kv.second.waves, kv.second.graph_steps, kv.second.ms);
    s << " \"" << kv.first << "\": " << buf << (++k < m.size() ? ",\n" : "\n");
  }
  s << "}\n";
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << s.str();
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace dg2
