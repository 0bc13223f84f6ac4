// internal.h -- shared host-side declarations of the topsimp library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/topsimp.h"

namespace ts {

// Error carrying a TS_* status code.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define TS_HIP(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      throw ::ts::Error(e_ == hipErrorOutOfMemory ? TS_ERR_OOM : TS_ERR_HIP,    \
                        std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Device workspace: named grow-only buffers owned by the context.
struct Workspace {
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  std::map<std::string, Buf> host_bufs;  // pinned host staging (hipHostMalloc)
  void* get(const std::string& name, size_t bytes);
  template <class T>
  T* get(const std::string& name, size_t count) {
    return static_cast<T*>(get(name, count * sizeof(T) + 16));
  }
  // Pinned host memory for device-to-host copies at full link speed.
  void* host(const std::string& name, size_t bytes);
  template <class T>
  T* host(const std::string& name, size_t count) {
    return static_cast<T*>(host(name, count * sizeof(T) + 16));
  }
  void release();
  size_t total_bytes() const;
};

// Launch-parameter autotuning.  For each key (a stage and a size class) the
// first calls try the candidates in turn and report their time; later calls
// get the fastest.  Only parameters that leave results unchanged are tuned.
struct Tuner {
  struct Entry {
    std::vector<double> seconds;  // per candidate, < 0 until tried
    int best = -1;
  };
  std::map<std::string, Entry> entries;
  // Index of the candidate to use now (ncand > 0).
  int pick(const std::string& key, int ncand) {
    Entry& e = entries[key];
    if (e.seconds.empty()) e.seconds.assign(ncand, -1.0);
    if (e.best >= 0) return e.best;
    for (int i = 0; i < ncand; ++i)
      if (e.seconds[i] < 0) return i;
    return 0;
  }
  void report(const std::string& key, int idx, double secs) {
    Entry& e = entries[key];
    if (e.best >= 0 || idx < 0 || idx >= int(e.seconds.size())) return;
    e.seconds[idx] = secs;
    int b = -1;
    for (int i = 0; i < int(e.seconds.size()); ++i) {
      if (e.seconds[i] < 0) return;  // not all tried yet
      if (b < 0 || e.seconds[i] < e.seconds[b]) b = i;
    }
    e.best = b;
  }
};

// Per-stage device timing with HIP events on the context stream.
struct Timer {
  hipStream_t stream = nullptr;
  bool enabled = true;
  std::vector<std::string> names;
  std::vector<hipEvent_t> begin, end;
  std::vector<std::string> open;
  void reset();
  void start(const std::string& name);
  void stop();
  // Accumulated ms per stage name (in first-seen order).
  void collect(std::vector<std::string>* names_out, std::vector<double>* ms_out);
  void destroy();
};

struct Grid {
  int Lx, Ly, Lz;
  int n;
};

// Slices of one device area handed out in order (256-byte aligned), for
// code that must not allocate; running past the area is an argument error.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  template <class T>
  T* get(const std::string&, size_t count) {
    const size_t at = (used + 255) & ~size_t(255);
    const size_t bytes = count * sizeof(T) + 16;
    if (at + bytes > cap) throw Error(TS_ERR_ARG, "scratch area too small for this size");
    used = at + bytes;
    return reinterpret_cast<T*>(base + at);
  }
};

// Sorting and scanning primitives (sort.hip).
void scan_exclusive_u32(Workspace& ws, const uint32_t* in, uint32_t* out, size_t n,
                        hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on bits [begin_bit, end_bit).
// The result is left in keys/vals; tmp buffers are taken from the workspace.
void radix_sort_u64(Workspace& ws, uint64_t* keys, uint32_t* vals, size_t n, int begin_bit,
                    int end_bit, hipStream_t s);
void radix_sort_u32(Workspace& ws, uint32_t* keys, uint32_t* vals, size_t n, int begin_bit,
                    int end_bit, hipStream_t s);
// The same sort with its temporary buffers taken from an arena.
void radix_sort_u32(Arena& arena, uint32_t* keys, uint32_t* vals, size_t n, int begin_bit,
                    int end_bit, hipStream_t s);

}  // namespace ts

struct ts_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  ts::Workspace ws;
  ts::Timer timer;
  ts::Tuner tuner;
  std::vector<std::string> stage_names_store;
  std::vector<const char*> stage_names;
  std::vector<double> stage_ms;
  std::vector<std::string> tuner_keys_store;
  std::vector<const char*> tuner_keys;
  std::vector<int> tuner_choices;
};
