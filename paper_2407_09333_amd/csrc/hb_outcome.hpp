// hb_outcome.hpp -- a request's final status and the text explaining it, recorded on
// whichever thread fails the request (a staging thread, the serving loop) and handed to the
// thread that asks for the result.  The library's error text is per thread, so without
// this the caller of wait/poll would see the status but not why.  Free of HIP calls, so
// the host can check it on its own.
#pragma once

#include <string>

namespace hb {

struct Outcome {
    int status = 0;    // HB_OK until the first failure
    std::string text;  // that failure's explanation

    // Record a failure; the first one wins (later ones are its consequences).
    void fail(int st, const std::string &why)
    {
        if (status != 0 || st == 0) return;
        status = st;
        text = why.empty() ? std::string("request failed") : why;
    }

    // On the asking thread: give a failed outcome's text to `set_error(status, text)`,
    // the library's per-thread error slot.  Returns the status.
    template <class SetError>
    int deliver(SetError &&set_error) const
    {
        if (status != 0) set_error(status, text);
        return status;
    }
};

}  // namespace hb
