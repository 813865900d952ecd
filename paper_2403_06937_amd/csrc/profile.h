// Optional kernel timing: hipEvent pairs around the product kernels.
#pragma once
#include "common.h"

namespace tcm {

bool profile_enabled();
// While suspended (e.g. during hipGraph capture) no events are recorded.
void profile_suspend(bool on);
// Records an event on s before the launch (begin) and after it (end).
void profile_begin(int kind, hipStream_t s);
void profile_end(int kind, hipStream_t s);

struct ProfileScope {
  int kind;
  hipStream_t s;
  bool on;
  ProfileScope(int k, hipStream_t st) : kind(k), s(st), on(profile_enabled()) {
    if (on) profile_begin(kind, s);
  }
  ~ProfileScope() {
    if (on) profile_end(kind, s);
  }
};

}  // namespace tcm
