// Error translation at the C ABI: every exported function runs its body
// through capi_guard, which maps exceptions to rfd_status codes and stores the
// message for rfd_last_error().
#pragma once

#include <exception>
#include <new>
#include <string>

#include "rfd_common.hpp"

namespace rfd {

std::string& last_error_slot();

template <typename F>
int capi_guard(F&& f) {
  try {
    last_error_slot().clear();
    f();
    return ST_OK;
  } catch (const Error& e) {
    last_error_slot() = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    last_error_slot() = "host allocation failed";
    return ST_ENOMEM;
  } catch (const std::exception& e) {
    last_error_slot() = e.what();
    return ST_EINVAL;
  } catch (...) {
    last_error_slot() = "unknown error";
    return ST_EINVAL;
  }
}

}  // namespace rfd
