// tsf_internal.h -- helpers shared by the translation units of libtsf.
#pragma once
#include "../../include/tsf.h"

// Record the reason of an error for tsf_last_error() and return `st`.
tsf_status tsf_fail(tsf_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
