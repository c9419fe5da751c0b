// Internal to libfciqmc: shared error reporting of its translation units.
#pragma once

// Record the message fciqmc_last_error() returns for this thread and return
// `code` (printf-style formatting).
int fq_set_error(int code, const char* fmt, ...);
