// spect_internal.h - shared by the host translation units of the library.
#pragma once

namespace spect_internal {
// Set the thread's spect_last_error() message and return code.
int set_error(int code, const char *msg);
// Clear the message and return SPECT_OK.
int clear_error();
}  // namespace spect_internal
