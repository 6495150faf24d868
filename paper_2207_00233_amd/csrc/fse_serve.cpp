// fse_serve.cpp -- asynchronous serving entry points (fse_submit / fse_poll).
#include "fse_internal.h"

namespace fse {

int serving_init(fse_plan_s*) { return FSE_OK; }
void serving_shutdown(fse_plan_s*) {}

}  // namespace fse

extern "C" {

int32_t fse_submit(fse_plan_t pl, const fse_frame* frame, uint64_t* ticket) {
  if (!pl || !frame || !ticket) return FSE_ERR_INVALID;
  return FSE_ERR_UNSUPPORTED;
}

int32_t fse_poll(fse_plan_t pl, uint64_t, int32_t) {
  if (!pl) return FSE_ERR_INVALID;
  return FSE_ERR_TICKET;
}

}  // extern "C"
