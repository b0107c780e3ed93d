// Batched form of a multi-instance plan (filled in by the persistent gridder).
#include "internal.h"

namespace mwg {

Status batch_prepare(Plan &P, hipStream_t s) {
    (void)s;
    P.batch = nullptr;
    return Status::Ok();
}

Status batch_grid(Plan &, const void *const *, const void *const *, void *const *, int, hipStream_t) {
    return make_error(MW_ERR_STATE, "batched form not prepared");
}

Status batch_degrid(Plan &, const void *const *, const void *const *, const void *const *,
                    void *const *, void *const *, hipStream_t) {
    return make_error(MW_ERR_STATE, "batched form not prepared");
}

void batch_release(Plan &P) { P.batch = nullptr; }

} // namespace mwg
