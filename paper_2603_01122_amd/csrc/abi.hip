// abi.hip -- error reporting and device queries of the C ABI.
#include "common.hpp"

namespace capred {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

cap_status fail(cap_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

cap_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return CAP_E_HIP;
}

}  // namespace capred

extern "C" int32_t cap_abi_version(void) { return CAP_ABI_VERSION; }

extern "C" const char* cap_last_error(void) { return capred::g_last_error.c_str(); }

extern "C" int32_t cap_device_cu_count(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}
