// Error type and argument checks of the library.  Host code only, with no
// HIP dependency, so that the weight-file parser and the planner can also be
// built and checked on their own.
#pragma once

#include <string>

namespace td {

struct Error {
  int status;
  std::string msg;
};

#define TD_CHECK(cond, status, msg)                                           \
  do {                                                                        \
    if (!(cond)) throw ::td::Error{(status), (msg)};                          \
  } while (0)

}  // namespace td
