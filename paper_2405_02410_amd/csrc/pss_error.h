// The thread-local error message behind pss_last_error, shared by the
// translation units of the host library.
#pragma once

#include <cstdarg>

#include "../../include/pss.h"

namespace pss_internal {
// format the message, store it for pss_last_error, return code
pss_status set_error(pss_status code, const char* fmt, va_list ap);
}  // namespace pss_internal
