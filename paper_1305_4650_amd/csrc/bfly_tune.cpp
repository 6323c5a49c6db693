// Tuning table of the autotuner (bfly_tune): the launch shapes measured
// fastest for one apply, keyed by device name, d, q, N (as log2 N), nrhs,
// precision, phase id and direction.  With BFLY_TUNE_CACHE set, the table is
// read from that JSON file at the first lookup and written back after each
// store (one object per record, in a flat "records" array).
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "bfly_internal.h"

namespace bfly {
namespace {

using Key = std::tuple<std::string, int, int, int, int, int, int, int>;  // dev, d, q, L, nrhs, prec, phase, adj

struct Rec {
  TuneParams p;
  double ms = 0.0;
};

struct Table {
  std::mutex mu;
  bool loaded = false;
  std::map<Key, Rec> rec;
  std::map<int, std::string> dev_name;  // device index -> name
};

Table& table() {
  static Table t;
  return t;
}

const char* cache_path() {
  const char* p = getenv("BFLY_TUNE_CACHE");
  return p && *p ? p : nullptr;
}

// name of the current device (gcnArchName plus marketing name), cached
std::string current_device(Table& t) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  auto it = t.dev_name.find(dev);
  if (it != t.dev_name.end()) return it->second;
  hipDeviceProp_t prop;
  std::string name = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    name = std::string(prop.gcnArchName) + " " + prop.name;
    for (char& c : name)
      if (c == '"' || c == '\\' || (unsigned char)c < 32) c = ' ';
  }
  t.dev_name[dev] = name;
  return name;
}

// ---- minimal JSON reading for the records this file writes ----
struct Reader {
  const std::string& s;
  size_t i = 0;
  void ws() {
    while (i < s.size() && isspace((unsigned char)s[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\' && i + 1 < s.size()) ++i;
      out->push_back(s[i++]);
    }
    if (i >= s.size()) return false;
    ++i;
    return true;
  }
  bool num(double* out) {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    *out = strtod(b, &e);
    if (e == b) return false;
    i += (size_t)(e - b);
    return true;
  }
};

// one record object: {"device": "...", "d": 2, ..., "split": [2, 2, 1]}
bool read_record(Reader& r, Key* k, Rec* v) {
  if (!r.eat('{')) return false;
  std::string dev;
  double d = -1, q = -1, L = -1, nrhs = -1, prec = -1, ph = -1, adj = -1;
  for (bool first = true;; first = false) {
    if (r.eat('}')) break;
    if (!first && !r.eat(',')) return false;
    std::string name;
    if (!r.str(&name) || !r.eat(':')) return false;
    if (name == "device") {
      if (!r.str(&dev)) return false;
    } else if (name == "split") {
      if (!r.eat('[')) return false;
      v->p.nsplit = 0;
      for (bool f2 = true;; f2 = false) {
        if (r.eat(']')) break;
        if (!f2 && !r.eat(',')) return false;
        double x;
        if (!r.num(&x)) return false;
        if (v->p.nsplit < 16) v->p.split[v->p.nsplit++] = (int)x;
      }
    } else {
      double x;
      if (!r.num(&x)) return false;
      if (name == "d") d = x;
      else if (name == "q") q = x;
      else if (name == "log2N") L = x;
      else if (name == "nrhs") nrhs = x;
      else if (name == "prec") prec = x;
      else if (name == "phase") ph = x;
      else if (name == "adjoint") adj = x;
      else if (name == "ub_first") v->p.ub_first = (int)x;
      else if (name == "ub_second") v->p.ub_second = (int)x;
      else if (name == "rc_one") v->p.rc_one = (int)x;
      else if (name == "ms") v->ms = x;
    }
  }
  if (dev.empty() || d < 0 || q < 0 || L < 0 || nrhs < 0 || prec < 0 || ph < 0 || adj < 0) return false;
  *k = Key(dev, (int)d, (int)q, (int)L, (int)nrhs, (int)prec, (int)ph, (int)adj);
  return true;
}

void load(Table& t) {
  t.loaded = true;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = fopen(path, "rb");
  if (!f) return;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  fclose(f);
  // the records array: a malformed file is ignored from the first bad record on
  const size_t a = s.find("\"records\"");
  if (a == std::string::npos) return;
  Reader r{s, a + 9};
  if (!r.eat(':') || !r.eat('[')) return;
  for (bool first = true;; first = false) {
    if (r.eat(']')) break;
    if (!first && !r.eat(',')) return;
    Key k;
    Rec v;
    if (!read_record(r, &k, &v)) return;
    t.rec[k] = v;
  }
}

hipError_t save(const Table& t) {
  const char* path = cache_path();
  if (!path) return hipSuccess;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return hipErrorFileNotFound;
  fprintf(f, "{\"version\": 1, \"records\": [");
  bool first = true;
  for (const auto& kv : t.rec) {
    const Key& k = kv.first;
    const Rec& v = kv.second;
    fprintf(f, "%s\n  {\"device\": \"%s\", \"d\": %d, \"q\": %d, \"log2N\": %d, \"nrhs\": %d, \"prec\": %d, "
               "\"phase\": %d, \"adjoint\": %d, \"ub_first\": %d, \"ub_second\": %d, \"rc_one\": %d, \"split\": [",
            first ? "" : ",", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
            std::get<5>(k), std::get<6>(k), std::get<7>(k), v.p.ub_first, v.p.ub_second, v.p.rc_one);
    for (int i = 0; i < v.p.nsplit; ++i) fprintf(f, "%s%d", i ? ", " : "", v.p.split[i]);
    fprintf(f, "], \"ms\": %.6g}", v.ms);
    first = false;
  }
  fprintf(f, "\n]}\n");
  const bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), path) != 0) return hipErrorFileNotFound;
  return hipSuccess;
}

}  // namespace

bool tune_lookup(const Geo& g, int nrhs, int prec, TuneParams* p) {
  Table& t = table();
  std::lock_guard<std::mutex> lk(t.mu);
  if (!t.loaded) load(t);
  if (t.rec.empty()) return false;
  const Key k(current_device(t), g.d, g.q, g.L, nrhs, prec, g.phase, g.adj);
  auto it = t.rec.find(k);
  if (it == t.rec.end()) return false;
  *p = it->second.p;
  return true;
}

hipError_t tune_store(const Geo& g, int nrhs, int prec, const TuneParams& p, double ms) {
  Table& t = table();
  std::lock_guard<std::mutex> lk(t.mu);
  if (!t.loaded) load(t);
  const Key k(current_device(t), g.d, g.q, g.L, nrhs, prec, g.phase, g.adj);
  t.rec[k] = Rec{p, ms};
  return save(t);
}

void tune_clear() {
  Table& t = table();
  std::lock_guard<std::mutex> lk(t.mu);
  t.rec.clear();
  t.loaded = false;  // the cache file's records come back at the next lookup
}

}  // namespace bfly
