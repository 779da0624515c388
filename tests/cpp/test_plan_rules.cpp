// Host-side checks of the launch-plan rules (dry run, no GPU): every fork of
// a plan starts from lane 0 and every join ends on it, and a plan on a fixed
// scratch buffer stays on one lane.  Prints "ok" and returns 0 on success.
#include <cstdio>
#include <cstdlib>

#include "library.h"

using qtt::Plan;

static int failures = 0;

template <class F>
static void expect_error(const char* what, F&& f) {
  try {
    f();
    std::printf("FAIL: %s did not raise\n", what);
    ++failures;
  } catch (const qtt::Error&) {
  }
}

int main() {
  setenv("QTTPDF_DRYRUN", "1", 1);
  {
    Plan p;  // a fork from lane 0 and a join back are allowed
    p.fork(3);
    p.on(1);
    p.on(2);
    p.join(3);
  }
  expect_error("fork from a lane other than 0", [] {
    Plan p;
    p.fork(2);
    p.on(1);
    p.fork(2);
  });
  expect_error("fork on a plan with a fixed scratch buffer", [] {
    static double buf[64];
    Plan p;
    p.arena = buf;
    p.arena_cap = 64;
    p.fork(2);
  });
  expect_error("arena overrun", [] {
    static double buf[64];
    Plan p;
    p.arena = buf;
    p.arena_cap = 64;
    p.alloc(40);
    p.alloc(40);
  });
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
