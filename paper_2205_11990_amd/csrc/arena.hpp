// Device memory arena: stack-like sub-allocation out of large hipMalloc'd
// chunks that are kept for the lifetime of the owning state, so that steady
// state time stepping performs no device allocation at all.
//
// For lock-step instances (see Lanes) each chunk is allocated once for all
// of them, chunk_bytes per instance: instance i's copy of any buffer lies
// i * chunk_bytes after instance 0's, the same stride in every arena that
// shares the chunk size.  A request larger than one chunk would break that
// stride and is refused then.
#pragma once
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace mpsv {

class Arena {
 public:
  struct Mark {
    size_t chunk, off;
  };

  explicit Arena(size_t chunk_bytes = (size_t)256 << 20, int instances = 1)
      : chunk_(chunk_bytes), inst_(instances < 1 ? 1 : instances) {}
  // An arena over a caller's device buffer: never allocates, and a request
  // beyond the buffer fails with kEnomem.
  Arena(void* base, size_t bytes) : chunk_(bytes), inst_(1), fixed_(true) {
    chunks_.push_back({base, bytes});
  }
  ~Arena() { release_all(); }
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;

  // 256-byte aligned allocation of n doubles (n may be 0).
  double* alloc(size_t n) { return (double*)alloc_bytes(n * sizeof(double)); }
  int* alloc_int(size_t n) { return (int*)alloc_bytes(n * sizeof(int)); }

  void* alloc_bytes(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    while (cur_ < chunks_.size()) {
      if (off_ + bytes <= chunks_[cur_].size) {
        void* p = (char*)chunks_[cur_].ptr + off_;
        off_ += bytes;
        note_peak();
        return p;
      }
      ++cur_;
      off_ = 0;
    }
    if (fixed_)
      throw Error(kEnomem, "fixed scratch of " + std::to_string(chunk_) +
                               " bytes exhausted by a request of " +
                               std::to_string(bytes) + " bytes");
    if (inst_ > 1 && bytes > chunk_)
      throw Error(kEnomem, "device arena: a request of " + std::to_string(bytes) +
                               " bytes exceeds the per-instance chunk of " +
                               std::to_string(chunk_) + " bytes");
    size_t sz = bytes > chunk_ ? bytes : chunk_;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sz * (size_t)inst_);
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      throw Error(kEnomem, "device arena: hipMalloc of " +
                               std::to_string(sz * (size_t)inst_) + " bytes failed");
    }
    chunks_.push_back({p, sz});
    cur_ = chunks_.size() - 1;
    off_ = bytes;
    note_peak();
    return p;
  }

  Mark mark() const { return Mark{cur_, off_}; }
  void release(Mark m) {
    cur_ = m.chunk;
    off_ = m.off;
  }
  void reset() {
    cur_ = 0;
    off_ = 0;
  }
  // largest extent ever in use: whole chunks before the current one plus
  // the offset into it (chunk tails skipped by a larger request count too)
  size_t peak_bytes() const { return peak_; }
  // all instances together
  size_t reserved_bytes() const {
    size_t t = 0;
    for (auto& c : chunks_) t += c.size;
    return t * (size_t)inst_;
  }
  // largest single request (one chunk for lock-step instances)
  size_t max_alloc_bytes() const {
    if (fixed_) return chunks_[0].size > off_ ? chunks_[0].size - off_ : 0;
    return inst_ > 1 ? chunk_ : SIZE_MAX;
  }
  int instances() const { return inst_; }
  // bytes between two instances' copies of a buffer
  long instance_stride() const { return (long)chunk_; }
  // whether p points into instance 0's part of a chunk of this arena
  bool owns(const void* p) const {
    const char* c = static_cast<const char*>(p);
    for (auto& k : chunks_) {
      const char* b = static_cast<const char*>(k.ptr);
      if (c >= b && c < b + k.size) return true;
    }
    return false;
  }
  void release_all() {
    if (fixed_) {
      cur_ = 0;
      off_ = 0;
      return;
    }
    for (auto& c : chunks_) (void)hipFree(c.ptr);
    chunks_.clear();
    cur_ = 0;
    off_ = 0;
  }

 private:
  struct Chunk {
    void* ptr;
    size_t size;
  };
  void note_peak() {
    size_t used = off_;
    for (size_t i = 0; i < cur_; ++i) used += chunks_[i].size;
    if (used > peak_) peak_ = used;
  }
  std::vector<Chunk> chunks_;
  size_t chunk_;
  int inst_;
  bool fixed_ = false;
  size_t cur_ = 0, off_ = 0, peak_ = 0;
};

// RAII scope: everything allocated inside is released at scope exit.
class ArenaScope {
 public:
  explicit ArenaScope(Arena& a) : a_(a), m_(a.mark()) {}
  ~ArenaScope() { a_.release(m_); }

 private:
  Arena& a_;
  Arena::Mark m_;
};

}  // namespace mpsv
