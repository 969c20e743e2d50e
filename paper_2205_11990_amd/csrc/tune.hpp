// Launch-shape table.
//
// Some launches have several kernel variants that compute bit-identical
// results: they differ only in how the same arithmetic is spread over
// workgroups and waves (the output tile of the FP64 GEMM; the number of
// columns one wave carries through a reflector application, and whether the
// reflectors reach the waves from L2 or shared through LDS).  Which one is
// fastest depends on the exact shape and on how many lock-step instances a
// launch covers.  The table maps (knob, exact shape, instance class) to a
// variant; an offline tuner (paper_2205_11990_amd/tune.py) times the
// variants on the device inside real steps and writes the table, and the
// library loads it once, from MPSV_TUNING or else from tuning_gfx950.txt
// next to the shared library (MPSV_TUNING=none: no table).  A shape without
// an entry takes the built-in rule.  Since every variant gives the same
// bits, the table changes speed only, never a result.
//
// Table text: one entry per line, seven integers
//   knob a b c d class value
// ('#' starts a comment line).  The key integers per knob:
//   kTuneGemmTile   a = M, b = N, c = K, d = 4 * batch + 2 * a_kfast + b_nfast
//   kTuneApplyCols  a = rows, b = reflectors, c = columns, d = 2 * chunks + trans
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"

namespace mpsv {

enum TuneKnob : int32_t {
  kTuneGemmTile = 1,   // 0: 64 x 64 output tiles, 1: 128 x 128, 2: 128 x 64
  kTuneApplyCols = 2,  // columns per wave: 1, 2 or 4; LDS-shared: 8 + 1 or 2;
                       // LDS-shared with staged columns: 16 + 1 or 2
};

constexpr int kTuneKeyInts = 6;
struct TuneKey {
  int32_t v[kTuneKeyInts];  // knob, a, b, c, d, instance class
};

// Class of the number of lock-step instances a launch covers:
// 0: 1, 1: 2..7, 2: 8..31, 3: 32 or more.
int32_t tune_inst_class(long n);

struct TunePick {
  int value;  // the variant to launch
  int slot;   // timing slot while recording, else -1
};

// The table's value for `key` when it has one and bit `value` of `allowed`
// is set, else `dflt`.  While recording, the key is noted (with the value
// returned and the allowed set) and the launch that follows is timed with
// HIP events on `s`: call tune_end(s, slot) right after it.
TunePick tune_pick(hipStream_t s, const TuneKey& key, int dflt, uint32_t allowed);
void tune_end(hipStream_t s, int slot);

// Table management (the C-ABI mpsb_tune_* calls).
void tune_clear();
void tune_set(const TuneKey& key, int32_t value);  // value < 0: erase
bool tune_get(const TuneKey& key, int32_t* value);
long tune_size();
void tune_load(const std::string& path);  // replaces the table; kEinval on bad text
void tune_save(const std::string& path);
// Loads the default table once (MPSV_TUNING or the file next to the
// library); later calls do nothing.  Called before the first lookup.
void tune_load_default();

// Recording: on clears earlier records.  A record aggregates the launches
// of one key: the value used last, the allowed set, the launch count and
// their summed event time (read synchronises the device).
struct TuneRecord {
  TuneKey key;
  int32_t value;
  uint32_t allowed;
  int64_t launches;
  double ms;
};
void tune_record(bool on);
std::vector<TuneRecord> tune_records();

}  // namespace mpsv
