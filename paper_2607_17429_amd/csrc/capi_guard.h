// Exception -> status translation shared by the C entry points.
#pragma once

#include <new>
#include <stdexcept>

#include "common.h"

namespace ftlm {

// Runs f; an Error becomes its status code, anything else INVALID_ARG or
// OUT_OF_MEMORY, with the message stored for ftlm_last_error().
template <typename F>
int guarded(F&& f) {
  try {
    f();
    return FTLM_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host out of memory");
    return FTLM_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return FTLM_ERR_INVALID_ARG;
  }
}

}  // namespace ftlm
