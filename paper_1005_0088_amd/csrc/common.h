// Internal helpers shared by the host-side sources of the ndrho library.
#pragma once
#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/ndrho.h"

namespace ndrho {

// Internal error carrying an ndrho status code; converted to a return value
// at the C interface, never thrown across it.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

}  // namespace ndrho
