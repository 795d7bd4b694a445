// Optional per-launch kernel timing (see prof.cpp).
#pragma once

#include "common.h"

namespace ah {

extern bool g_prof;

struct ProfScope {
  bool active = false;
  std::string tag;
  hipStream_t st = nullptr;
  double bytes = 0.0;
  hipEvent_t a = nullptr, b = nullptr;
};

void prof_begin(ProfScope& s, const char* tag, hipStream_t st, double bytes);
void prof_end(ProfScope& s);

}  // namespace ah
