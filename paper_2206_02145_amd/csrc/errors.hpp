// errors.hpp -- the calling thread's last error message, shared by every translation unit of the
// library (lbcg_last_error returns it).
#pragma once

#include <string>

namespace lbcg {
inline std::string& last_error_slot() {
    static thread_local std::string s;
    return s;
}
}  // namespace lbcg
