#include "tune.hpp"

#include <dlfcn.h>

#include <array>
#include <atomic>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <sstream>

namespace mpsv {

namespace {

using Key = std::array<int32_t, kTuneKeyInts>;

Key key_of(const TuneKey& k) {
  Key a;
  for (int i = 0; i < kTuneKeyInts; ++i) a[i] = k.v[i];
  return a;
}

std::shared_mutex g_table_mu;
std::map<Key, int32_t> g_table;

std::once_flag g_default_once;

// recording
std::mutex g_rec_mu;
std::atomic<bool> g_recording{false};
struct Rec {
  int32_t value;
  uint32_t allowed;
  std::vector<int> slots;
};
std::map<Key, Rec> g_rec;
std::vector<hipEvent_t> g_ev;  // pairs: 2*slot, 2*slot+1
size_t g_used = 0;

bool known_knob(int32_t k) { return k == kTuneGemmTile || k == kTuneApplyCols; }

std::map<Key, int32_t> parse(const std::string& path) {
  std::ifstream in(path);
  MPSV_CHECK(in.good(), kEinval, "tuning table: cannot read " + path);
  std::map<Key, int32_t> t;
  std::string line;
  int ln = 0;
  while (std::getline(in, line)) {
    ++ln;
    const size_t b = line.find_first_not_of(" \t\r");
    if (b == std::string::npos || line[b] == '#') continue;
    std::istringstream ss(line);
    long v[kTuneKeyInts + 1];
    for (int i = 0; i <= kTuneKeyInts; ++i)
      MPSV_CHECK(static_cast<bool>(ss >> v[i]), kEinval,
                 "tuning table " + path + ": line " + std::to_string(ln) +
                     " needs seven integers");
    std::string rest;
    MPSV_CHECK(!(ss >> rest), kEinval,
               "tuning table " + path + ": extra text on line " + std::to_string(ln));
    MPSV_CHECK(known_knob((int32_t)v[0]), kEinval,
               "tuning table " + path + ": unknown knob on line " + std::to_string(ln));
    Key k;
    for (int i = 0; i < kTuneKeyInts; ++i) {
      MPSV_CHECK(v[i] >= 0 && v[i] <= INT32_MAX, kEinval,
                 "tuning table " + path + ": value out of range on line " +
                     std::to_string(ln));
      k[i] = (int32_t)v[i];
    }
    MPSV_CHECK(v[kTuneKeyInts] >= 0 && v[kTuneKeyInts] < 32, kEinval,
               "tuning table " + path + ": bad choice on line " + std::to_string(ln));
    t[k] = (int32_t)v[kTuneKeyInts];
  }
  return t;
}

std::string default_path() {
  const char* e = std::getenv("MPSV_TUNING");
  if (e && *e) return std::string(e) == "none" ? std::string() : std::string(e);
  // the table next to this shared library
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&tune_inst_class), &info) == 0 || !info.dli_fname)
    return std::string();
  std::string lib(info.dli_fname);
  const size_t cut = lib.find_last_of('/');
  const std::string dir = cut == std::string::npos ? std::string(".") : lib.substr(0, cut);
  const std::string path = dir + "/tuning_gfx950.txt";
  std::ifstream probe(path);
  return probe.good() ? path : std::string();
}

}  // namespace

int32_t tune_inst_class(long n) {
  if (n <= 1) return 0;
  if (n < 8) return 1;
  if (n < 32) return 2;
  return 3;
}

void tune_load_default() {
  std::call_once(g_default_once, [] {
    const std::string p = default_path();
    if (p.empty()) return;
    auto t = parse(p);
    std::unique_lock<std::shared_mutex> lk(g_table_mu);
    g_table = std::move(t);
  });
}

TunePick tune_pick(hipStream_t s, const TuneKey& key, int dflt, uint32_t allowed) {
  tune_load_default();
  const Key k = key_of(key);
  int v = dflt;
  {
    std::shared_lock<std::shared_mutex> lk(g_table_mu);
    auto it = g_table.find(k);
    if (it != g_table.end() && it->second < 32 && ((allowed >> it->second) & 1u))
      v = it->second;
  }
  TunePick p{v, -1};
  if (!g_recording.load(std::memory_order_relaxed)) return p;
  std::lock_guard<std::mutex> lk(g_rec_mu);
  if (!g_recording.load(std::memory_order_relaxed)) return p;
  if (2 * (g_used + 1) > g_ev.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      MPSV_HIP(hipEventCreate(&e));
      g_ev.push_back(e);
    }
  }
  p.slot = (int)g_used++;
  Rec& r = g_rec[k];
  r.value = v;
  r.allowed = allowed;
  r.slots.push_back(p.slot);
  MPSV_HIP(hipEventRecord(g_ev[2 * p.slot], s));
  return p;
}

void tune_end(hipStream_t s, int slot) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_rec_mu);
  MPSV_HIP(hipEventRecord(g_ev[2 * slot + 1], s));
}

void tune_clear() {
  tune_load_default();
  std::unique_lock<std::shared_mutex> lk(g_table_mu);
  g_table.clear();
}

void tune_set(const TuneKey& key, int32_t value) {
  MPSV_CHECK(known_knob(key.v[0]), kEinval, "tuning: unknown knob");
  for (int i = 0; i < kTuneKeyInts; ++i)
    MPSV_CHECK(key.v[i] >= 0, kEinval, "tuning: negative key integer");
  MPSV_CHECK(value < 32, kEinval, "tuning: choice out of range");
  tune_load_default();
  std::unique_lock<std::shared_mutex> lk(g_table_mu);
  if (value < 0)
    g_table.erase(key_of(key));
  else
    g_table[key_of(key)] = value;
}

bool tune_get(const TuneKey& key, int32_t* value) {
  tune_load_default();
  std::shared_lock<std::shared_mutex> lk(g_table_mu);
  auto it = g_table.find(key_of(key));
  if (it == g_table.end()) return false;
  if (value) *value = it->second;
  return true;
}

long tune_size() {
  tune_load_default();
  std::shared_lock<std::shared_mutex> lk(g_table_mu);
  return (long)g_table.size();
}

void tune_load(const std::string& path) {
  tune_load_default();
  auto t = parse(path);
  std::unique_lock<std::shared_mutex> lk(g_table_mu);
  g_table = std::move(t);
}

void tune_save(const std::string& path) {
  tune_load_default();
  std::ofstream out(path);
  MPSV_CHECK(out.good(), kEinval, "tuning table: cannot write " + path);
  out << "# knob a b c d class value\n";
  std::shared_lock<std::shared_mutex> lk(g_table_mu);
  for (const auto& e : g_table) {
    for (int i = 0; i < kTuneKeyInts; ++i) out << e.first[i] << ' ';
    out << e.second << '\n';
  }
  MPSV_CHECK(out.good(), kEinval, "tuning table: write failed for " + path);
}

void tune_record(bool on) {
  std::lock_guard<std::mutex> lk(g_rec_mu);
  g_recording.store(on);
  if (on) {
    g_rec.clear();
    g_used = 0;
  }
}

std::vector<TuneRecord> tune_records() {
  MPSV_HIP(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(g_rec_mu);
  std::vector<TuneRecord> out;
  out.reserve(g_rec.size());
  for (const auto& e : g_rec) {
    TuneRecord r;
    for (int i = 0; i < kTuneKeyInts; ++i) r.key.v[i] = e.first[i];
    r.value = e.second.value;
    r.allowed = e.second.allowed;
    r.launches = (int64_t)e.second.slots.size();
    r.ms = 0.0;
    for (int s : e.second.slots) {
      float t = 0.0f;
      MPSV_HIP(hipEventElapsedTime(&t, g_ev[2 * s], g_ev[2 * s + 1]));
      r.ms += t;
    }
    out.push_back(r);
  }
  return out;
}

}  // namespace mpsv
