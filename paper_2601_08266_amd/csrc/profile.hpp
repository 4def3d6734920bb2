// Per-kernel timing scopes (see profile.cpp).
#pragma once

#include "common.hpp"

namespace fsi {

bool profiling_enabled();

// Records a start event on construction and a stop event on destruction when
// timing is enabled; does nothing otherwise.
class ProfileScope {
  public:
    ProfileScope(const char *name, hipStream_t st);
    ~ProfileScope();
    ProfileScope(const ProfileScope &) = delete;
    ProfileScope &operator=(const ProfileScope &) = delete;

  private:
    hipStream_t st_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
    int slot_ = -1;
    bool active_ = false;
};

}  // namespace fsi
