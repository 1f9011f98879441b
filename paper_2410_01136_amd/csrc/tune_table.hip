// Launch shapes chosen by the autotuner, loaded from its cache file.
//
// The file is the tuner's JSON object: keys
//   "<device name>|<build id>|k<kernel>|f<field kind>|p<pixels>|n<steps>|q<freqs>[|g]"
// and values a lane count (1, 4, 16, 64) or [lane count, grid read mode 2|3].
// An entry applies to calls of that kernel family and field kind with exactly
// that many pixels, steps and frequencies, on a device of that name ("*":
// any device), and only if it was tuned on a library built from the same
// sources (build id).  Host code only.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tune_table.h"

#ifndef SYN_BUILD_ID
#define SYN_BUILD_ID "unversioned"
#endif

namespace sm {
namespace {

struct Entry {
  std::string device;
  int kernel, kind, lanes, grid_mode;  // grid_mode 0: none given
  long long npix, steps, freqs;
};

std::mutex g_mu;
std::vector<Entry> g_table;

// Minimal reader of the tuner's flat JSON object (string keys; integer or
// [integer, integer] values).  Any other shape is an error.
struct Reader {
  const std::string& s;
  size_t i = 0;
  std::string err;
  explicit Reader(const std::string& text) : s(text) {}
  void ws() {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
  }
  bool expect(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    err = std::string("expected '") + c + "' at byte " + std::to_string(i);
    return false;
  }
  bool peek(char c) {
    ws();
    return i < s.size() && s[i] == c;
  }
  bool string(std::string* out) {
    if (!expect('"')) return false;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      char c = s[i++];
      if (c == '\\') {
        if (i >= s.size()) break;
        const char e = s[i++];
        if (e == '"' || e == '\\' || e == '/') c = e;
        else {
          err = "unsupported escape in a key at byte " + std::to_string(i);
          return false;
        }
      } else if ((unsigned char)c < 0x20) {
        err = "control character in a key at byte " + std::to_string(i);
        return false;
      }
      out->push_back(c);
    }
    if (i >= s.size()) {
      err = "unterminated string";
      return false;
    }
    ++i;
    return true;
  }
  bool integer(long long* out) {
    ws();
    const size_t b = i;
    if (i < s.size() && s[i] == '-') ++i;
    while (i < s.size() && s[i] >= '0' && s[i] <= '9') ++i;
    if (i == b || (i == b + 1 && s[b] == '-') || i - b > 18) {
      err = "expected an integer at byte " + std::to_string(b);
      return false;
    }
    *out = std::strtoll(s.c_str() + b, nullptr, 10);
    return true;
  }
};

// Splits "dev|id|k0|f1|p786432|n512|q3[|g]" into its fields; false if malformed.
bool parse_key(const std::string& key, Entry* e, std::string* build_id, bool* grid_flag) {
  std::vector<std::string> parts;
  size_t b = 0;
  for (;;) {
    const size_t p = key.find('|', b);
    parts.push_back(key.substr(b, p == std::string::npos ? std::string::npos : p - b));
    if (p == std::string::npos) break;
    b = p + 1;
  }
  if (parts.size() != 7 && parts.size() != 8) return false;
  if (parts.size() == 8 && parts[7] != "g") return false;
  *grid_flag = parts.size() == 8;
  e->device = parts[0];
  *build_id = parts[1];
  const char tags[5] = {'k', 'f', 'p', 'n', 'q'};
  long long v[5];
  for (int k = 0; k < 5; ++k) {
    const std::string& f = parts[2 + k];
    if (f.size() < 2 || f[0] != tags[k]) return false;
    for (size_t j = 1; j < f.size(); ++j)
      if (f[j] < '0' || f[j] > '9') return false;
    if (f.size() > 13) return false;
    v[k] = std::strtoll(f.c_str() + 1, nullptr, 10);
  }
  e->kernel = (int)v[0];
  e->kind = (int)v[1];
  e->npix = v[2];
  e->steps = v[3];
  e->freqs = v[4];
  return e->kernel >= 0 && e->kernel <= 2 && e->kind >= 0 && e->kind <= 4 && e->npix >= 1 &&
         e->steps >= 1 && e->freqs >= 1;
}

// Name of the current device, cached per ordinal; empty without a device.
std::string current_device_name() {
  static std::mutex mu;
  static std::vector<std::string> names;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    (void)hipGetLastError();
    return std::string();
  }
  std::lock_guard<std::mutex> lk(mu);
  if ((int)names.size() <= dev) names.resize(dev + 1);
  if (names[dev].empty()) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
      (void)hipGetLastError();
      return std::string();
    }
    names[dev] = p.name;
  }
  return names[dev];
}

}  // namespace

const char* build_id() { return SYN_BUILD_ID; }

bool lanes_valid(long long kernel, long long lanes) {
  if (lanes == 8) return kernel == 0 || kernel == 1;  // forward and reverse marches only
  return lanes == 1 || lanes == 4 || lanes == 16 || lanes == 64;
}

bool tune_load(const char* path, int* kept, std::string* err) {
  FILE* f = std::fopen(path, "rb");
  if (f == nullptr) {
    *err = std::string("cannot open the tuning file ") + path;
    return false;
  }
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) {
    text.append(buf, n);
    if (text.size() > (64u << 20)) {
      std::fclose(f);
      *err = "tuning file larger than 64 MiB";
      return false;
    }
  }
  std::fclose(f);
  Reader r(text);
  std::vector<Entry> out;
  if (!r.expect('{')) {
    *err = "tuning file: " + r.err;
    return false;
  }
  bool first = true;
  while (!r.peek('}')) {
    if (!first && !r.expect(',')) {
      *err = "tuning file: " + r.err;
      return false;
    }
    first = false;
    std::string key, id;
    if (!r.string(&key) || !r.expect(':')) {
      *err = "tuning file: " + r.err;
      return false;
    }
    long long lanes = 0, mode = 0;
    if (r.peek('[')) {
      r.expect('[');
      if (!r.integer(&lanes) || !r.expect(',') || !r.integer(&mode) || !r.expect(']')) {
        *err = "tuning file: " + r.err;
        return false;
      }
      if (mode != 2 && mode != 3) {
        *err = "tuning file: grid read mode must be 2 or 3 (key " + key + ")";
        return false;
      }
    } else if (!r.integer(&lanes)) {
      *err = "tuning file: " + r.err;
      return false;
    }
    Entry e;
    bool grid_flag = false;
    if (!parse_key(key, &e, &id, &grid_flag) || grid_flag != (mode != 0)) {
      *err = "tuning file: malformed key " + key;
      return false;
    }
    if (!lanes_valid(e.kernel, lanes)) {
      *err = "tuning file: lane count must be 1, 4, 8, 16 or 64 (1, 4, 16 or 64 for the batch "
             "kernels; key " + key + ")";
      return false;
    }
    e.lanes = (int)lanes;
    e.grid_mode = (int)mode;
    if (id == build_id()) out.push_back(e);  // entries tuned on other sources are stale
  }
  r.expect('}');
  r.ws();
  if (r.i != text.size()) {
    *err = "tuning file: trailing bytes after the object";
    return false;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.swap(out);
  *kept = (int)g_table.size();
  return true;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

int tune_entries() {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int)g_table.size();
}

bool tune_lookup(int kernel, int kind, long long npix, long long steps, long long freqs,
                 int* lanes, int* grid_mode) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_table.empty()) return false;
  }
  const std::string dev = current_device_name();
  std::lock_guard<std::mutex> lk(g_mu);
  for (const Entry& e : g_table) {
    if (e.kernel != kernel || e.kind != kind || e.npix != npix || e.steps != steps ||
        e.freqs != freqs)
      continue;
    if (e.device != "*" && e.device != dev) continue;
    *lanes = e.lanes;
    *grid_mode = e.grid_mode;
    return true;
  }
  return false;
}

}  // namespace sm
