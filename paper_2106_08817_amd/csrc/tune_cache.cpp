// Persistent autotuning: a JSON file that maps "<gcnArchName>/<shape class>"
// to a plan's tuning choices, so that a plan of a class already timed on a
// device of the same architecture takes its choices without running.
//
// File format (written by this file, read back strictly; anything else is
// treated as an empty cache and replaced at the next store):
//   {
//     "format": "shoot-tune-1",
//     "entries": {
//       "gfx950:sramecc+:xnack-/d3-grad-v25-x7_8-r16-l2-f0": [0, 1, 0, 0, 0, 0]
//     }
//   }
#include "shoot.h"

#include <hip/hip_runtime.h>
#include <unistd.h>

#include <cctype>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "plan_access.h"

namespace {

constexpr const char* FORMAT = "shoot-tune-1";
using Entries = std::map<std::string, std::vector<long long>>;

// Recursive-descent reader of the subset of JSON the file uses: objects,
// arrays of integers, strings with the escapes \" \\ \/ \b \f \n \r \t.
struct Reader {
  const std::string& s;
  size_t i = 0;
  explicit Reader(const std::string& text) : s(text) {}

  void ws() {
    while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string& out) {
    if (!eat('"')) return false;
    out.clear();
    while (i < s.size()) {
      const char c = s[i++];
      if (c == '"') return true;
      if ((unsigned char)c < 0x20) return false;
      if (c != '\\') {
        out.push_back(c);
        continue;
      }
      if (i >= s.size()) return false;
      const char e = s[i++];
      switch (e) {
        case '"': out.push_back('"'); break;
        case '\\': out.push_back('\\'); break;
        case '/': out.push_back('/'); break;
        case 'b': out.push_back('\b'); break;
        case 'f': out.push_back('\f'); break;
        case 'n': out.push_back('\n'); break;
        case 'r': out.push_back('\r'); break;
        case 't': out.push_back('\t'); break;
        default: return false;
      }
    }
    return false;
  }
  bool integer(long long& v) {
    ws();
    const size_t b = i;
    if (i < s.size() && s[i] == '-') ++i;
    const size_t d = i;
    while (i < s.size() && std::isdigit((unsigned char)s[i])) ++i;
    if (i == d || i - d > 9) return false;
    v = std::stoll(s.substr(b, i - b));
    return true;
  }
  bool int_array(std::vector<long long>& out) {
    out.clear();
    if (!eat('[')) return false;
    if (eat(']')) return true;
    do {
      long long v = 0;
      if (!integer(v)) return false;
      out.push_back(v);
    } while (eat(','));
    return eat(']');
  }
  bool entries(Entries& out) {
    if (!eat('{')) return false;
    if (eat('}')) return true;
    do {
      std::string k;
      std::vector<long long> v;
      if (!str(k) || !eat(':') || !int_array(v)) return false;
      out[k] = v;
    } while (eat(','));
    return eat('}');
  }
  bool document(Entries& out) {
    if (!eat('{')) return false;
    bool fmt = false, ent = false;
    do {
      std::string k;
      if (!str(k) || !eat(':')) return false;
      if (k == "format" && !fmt) {
        std::string f;
        if (!str(f) || f != FORMAT) return false;
        fmt = true;
      } else if (k == "entries" && !ent) {
        if (!entries(out)) return false;
        ent = true;
      } else {
        return false;
      }
    } while (eat(','));
    if (!eat('}')) return false;
    ws();
    return fmt && ent && i == s.size();
  }
};

// The cache's entries; empty when the file is missing, unreadable or not in
// the format above.
Entries read_cache(const char* path) {
  Entries e;
  std::ifstream f(path, std::ios::binary);
  if (!f) return e;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  Reader r(text);
  if (!r.document(e)) e.clear();
  return e;
}

std::string quoted(const std::string& k) {
  std::string o = "\"";
  for (char c : k) {
    if (c == '"' || c == '\\') {
      o.push_back('\\');
      o.push_back(c);
    } else if ((unsigned char)c < 0x20) {
      char b[8];
      std::snprintf(b, sizeof(b), "\\u%04x", (unsigned)(unsigned char)c);
      o += b;
    } else {
      o.push_back(c);
    }
  }
  return o + "\"";
}

// Writes the entries to a temporary file beside `path` and renames it over
// `path`; false on any failure (the temporary file is removed).
bool write_cache(const char* path, const Entries& e) {
  std::string text = "{\n  \"format\": \"" + std::string(FORMAT) + "\",\n  \"entries\": {";
  bool first = true;
  for (const auto& kv : e) {
    text += first ? "\n    " : ",\n    ";
    first = false;
    text += quoted(kv.first) + ": [";
    for (size_t j = 0; j < kv.second.size(); ++j) text += (j ? ", " : "") + std::to_string(kv.second[j]);
    text += "]";
  }
  text += first ? "}\n}\n" : "\n  }\n}\n";
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

shoot_status cfail(shoot_status st, const std::string& msg) {
  shoot_internal_set_error(msg.c_str());
  return st;
}

}  // namespace

#pragma GCC visibility push(default)
extern "C" {

shoot_status shoot_autotune_cached(shoot_plan plan, const char* path, int32_t* hit, void* stream) {
  if (hit) *hit = 0;
  if (!plan || !path) return cfail(SHOOT_E_ARG, "NULL argument");
  int unfused = 0;
  const int dev = shoot_internal_device(plan, &unfused);
  if (dev < 0) return cfail(SHOOT_E_STATE, "plan is not bound to a workspace");
  if (unfused) return SHOOT_OK;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return cfail(SHOOT_E_HIP, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
  const std::string key = std::string(prop.gcnArchName) + "/" + shoot_internal_tune_class(plan);

  Entries cache = read_cache(path);
  auto it = cache.find(key);
  if (it != cache.end() && it->second.size() == SHOOT_TUNE_COUNT) {
    int32_t c[SHOOT_TUNE_COUNT];
    bool valid = true;
    for (int k = 0; k < SHOOT_TUNE_COUNT; ++k) {
      valid = valid && (it->second[k] == 0 || it->second[k] == 1);
      c[k] = (int32_t)it->second[k];
    }
    if (valid) {
      shoot_status st = shoot_plan_set_tuning(plan, c);
      if (st != SHOOT_OK) return st;
      if (hit) *hit = 1;
      return SHOOT_OK;
    }
  }
  shoot_status st = shoot_autotune(plan, stream);
  if (st != SHOOT_OK) return st;
  int32_t c[SHOOT_TUNE_COUNT];
  st = shoot_plan_get_tuning(plan, c);
  if (st != SHOOT_OK) return st;
  cache[key] = std::vector<long long>(c, c + SHOOT_TUNE_COUNT);
  if (!write_cache(path, cache)) return cfail(SHOOT_E_IO, std::string("cannot write the tuning cache ") + path);
  return SHOOT_OK;
}

}  // extern "C"
#pragma GCC visibility pop
