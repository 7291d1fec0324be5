// Per-kernel timing scopes (see profile.cpp).
#pragma once

#include <hip/hip_runtime.h>

namespace spg {

bool profiling();

class ProfScope {
 public:
  ProfScope(const char *name, hipStream_t st);
  ~ProfScope();
  ProfScope(const ProfScope &) = delete;
  ProfScope &operator=(const ProfScope &) = delete;

 private:
  const char *name_;
  hipStream_t st_;
  void *a_;
};

}  // namespace spg
