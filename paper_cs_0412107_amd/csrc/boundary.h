// Exceptions never cross the C boundary.  Every exported function that
// returns a status is a function-try-block; its handler calls
// exception_status(), which rethrows the exception in flight to classify it
// and reports it through the calling module's own error setter.  A host
// allocation sized by the caller's arguments (a huge n, an index list, a
// checkpoint's counts) or a worker thread that cannot start then returns a
// status instead of terminating the process.
#pragma once

#include <exception>
#include <new>
#include <stdexcept>
#include <string>

#include "../../include/mcinv.h"

namespace mcinv {

template <class Report>
mcinv_status exception_status(Report&& report) noexcept
{
    mcinv_status code = MCINV_EINTERNAL;
    try {
        try {
            throw;
        } catch (const std::bad_alloc&) {
            code = MCINV_ENOMEM;
            report(code, std::string("host memory allocation failed"));
        } catch (const std::length_error&) {
            code = MCINV_ENOMEM;
            report(code, std::string("a host buffer would exceed its size limit"));
        } catch (const std::exception& e) {
            report(code, std::string("unexpected host-side failure: ") + e.what());
        } catch (...) {
            report(code, std::string("unexpected host-side failure"));
        }
    } catch (...) {
        // the message itself could not be stored; the status still says what happened
    }
    return code;
}

}  // namespace mcinv
