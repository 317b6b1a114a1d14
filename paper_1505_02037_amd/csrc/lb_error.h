// lb_error.h -- the one per-thread error text behind lb_last_error(), shared
// by the handle and server halves of the C-ABI.
#ifndef LBNR_LB_ERROR_H
#define LBNR_LB_ERROR_H

namespace lbnr {

// Replaces this thread's last-error text (printf format).
void set_last_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

} // namespace lbnr

#endif
