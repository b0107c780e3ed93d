// C ABI of libmwagrid: argument validation, status codes, the thread-local error string and
// the plan lifecycle. Every entry point catches everything; nothing is thrown, printed or
// aborted across the boundary.
#include "internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>

// Scratch of the no-allocation gridding entry point (mw_grid_noalloc): the merge flush's
// partial tiles, in a file-scope device array instead of plan-owned memory. Every device the
// library runs on holds its own copy until the process ends; the host never uses the array's
// name as an address (it is a host-side stand-in), only the per-device address looked up with
// hipGetSymbolAddress below.
constexpr size_t kScratchBytes = size_t(192) << 20;
static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

// Plans of at least this many instances build them on parallel host threads.
constexpr int kParallelPlan = 4;

namespace {

thread_local std::string g_last_error;

// Per-device address of scratch, looked up once per device with that device current.
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// Live plans: a handle that was destroyed (or never made) is rejected instead of used.
std::mutex g_plans_mu;
std::set<void *> g_plans;

bool plan_is_live(mw_plan p) {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    return g_plans.count((void *)p) != 0;
}

mw_status fail(const mwg::Status &s) {
    g_last_error = s.msg;
    return s.code;
}

mw_status fail(mw_status code, const char *msg) {
    g_last_error = msg;
    return code;
}

mw_status ok() {
    g_last_error.clear();
    return MW_OK;
}

mwg::Status validate_instance(const mw_instance &d, int idx) {
    using mwg::make_error;
    auto bad = [&](const char *what) { return make_error(MW_ERR_INVALID_ARG, "instance %d: %s", idx, what); };
    if (d.nx < 8 || d.ny < 8 || (d.nx & 1) || (d.ny & 1)) return bad("nx and ny must be even and >= 8");
    if (d.nx > 4096 || d.ny > 4096)
        return make_error(MW_ERR_UNSUPPORTED, "instance %d: grids above 4096 are not supported", idx);
    if (!(d.du > 0.0) || !(d.dv > 0.0) || !std::isfinite(d.du) || !std::isfinite(d.dv))
        return bad("du and dv must be finite and > 0");
    if (d.nrow < 0 || d.nchan < 1) return bad("nrow must be >= 0 and nchan >= 1");
    if ((double)d.nrow * (double)d.nchan >= 2147483647.0)
        return make_error(MW_ERR_UNSUPPORTED, "instance %d: nrow * nchan must be < 2^31", idx);
    if (d.npol != 1 && d.npol != 2 && d.npol != 4) return bad("npol must be 1, 2 or 4");
    if (d.mem != MW_MEM_HOST && d.mem != MW_MEM_DEVICE) return bad("mem must be MW_MEM_HOST or MW_MEM_DEVICE");
    if (d.weighting < 0 || d.weighting > 2) return bad("weighting must be 0 (natural), 1 (uniform) or 2 (robust)");
    if (!std::isfinite(d.robust)) return bad("robust must be finite");
    if (!std::isfinite(d.wlo) || !std::isfinite(d.whi) || d.wlo > d.whi) return bad("need finite wlo <= whi");
    if (d.weighting != 0 && d.kernel_stack) return bad("density weighting is implemented for the built-in kernel");
    if (d.nrow > 0 && (!d.uvw_m || !d.freq_hz)) return bad("uvw_m and freq_hz are required");
    if ((d.ant1 == nullptr) != (d.ant2 == nullptr)) return bad("ant1 and ant2 go together");
    if (d.ant1 && (d.nant < 1 || d.nant > 65535)) return bad("nant must be in [1, 65535]");
    if (d.oversample < 1 || d.oversample > 16) return bad("oversample must be in [1, 16]");
    if (d.kernel_stack) {
        if (!d.kernel_offset || !d.kernel_support || !d.kernel_index || d.nkernel < 1 || d.kernel_elems < 1)
            return bad("kernel stacks need offsets, supports, per-group indices and nkernel >= 1");
    } else {
        if (d.support < 1 || d.support > 15 || (d.support % 2) == 0) return bad("support must be odd in [1, 15]");
    }
    return mwg::Status::Ok();
}

mwg::Status validate_tuning(const mw_tuning &t) {
    using mwg::make_error;
    if (t.tile != 0 && t.tile != 8 && t.tile != 16 && t.tile != 32 && t.tile != 64)
        return make_error(MW_ERR_INVALID_ARG, "tuning.tile must be 0, 8, 16, 32 or 64");
    if (t.split != 0 && t.split < 64) return make_error(MW_ERR_INVALID_ARG, "tuning.split must be 0 or >= 64");
    if (t.wg_waves != 0 && t.wg_waves != 1 && t.wg_waves != 2 && t.wg_waves != 4 && t.wg_waves != 8 &&
        t.wg_waves != 16)
        return make_error(MW_ERR_INVALID_ARG, "tuning.wg_waves must be 0, 1, 2, 4, 8 or 16");
    if (t.order < 0 || t.order > 3) return make_error(MW_ERR_INVALID_ARG, "tuning.order must be 0 ... 3");
    if (t.variant < 0 || t.variant > 6) return make_error(MW_ERR_INVALID_ARG, "tuning.variant must be 0..6");
    if (t.flush < 0 || t.flush > 3) return make_error(MW_ERR_INVALID_ARG, "tuning.flush must be 0 ... 3");
    if (t.schedule < 0 || t.schedule > 3) return make_error(MW_ERR_INVALID_ARG, "tuning.schedule must be 0 ... 3");
    return mwg::Status::Ok();
}

mwg::Status check_plan(mw_plan plan) {
    if (!plan) return mwg::make_error(MW_ERR_INVALID_ARG, "plan is NULL");
    if (!plan_is_live(plan)) return mwg::make_error(MW_ERR_STATE, "plan is not live (destroyed?)");
    mwg::Plan *P = (mwg::Plan *)plan;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != P->device)
        return mwg::make_error(MW_ERR_STATE, "current device %d is not the plan's device %d", dev, P->device);
    return mwg::Status::Ok();
}

void destroy_plan(mwg::Plan *P) {
    if (!P) return;
    (void)hipDeviceSynchronize();
    mwg::batch_release(*P);
    for (mwg::Instance *I : P->inst) {
        if (!I) continue;
        for (hipEvent_t &e : I->tev)
            if (e) (void)hipEventDestroy(e);
        if (I->src_ev) (void)hipEventDestroy(I->src_ev);
        if (I->src_h) (void)hipHostFree(I->src_h);
        mwg::image_release(*I);
        I->arena.release();
        delete I;
    }
    P->inst.clear();
    delete P;
}

} // namespace

namespace mwg {

Status static_scratch(void **ptr, size_t *bytes) {
    int dev = -1;
    MWG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return make_error(MW_ERR_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        MWG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return make_error(MW_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    *bytes = kScratchBytes;
    return Status::Ok();
}

} // namespace mwg


namespace {

mwg::Status check_inst(mw_plan plan, int32_t inst, mwg::Instance **out) {
    mwg::Status s = check_plan(plan);
    if (!s.ok()) return s;
    mwg::Plan *P = (mwg::Plan *)plan;
    if (inst < 0 || inst >= (int)P->inst.size()) return mwg::make_error(MW_ERR_INVALID_ARG, "inst out of range");
    *out = P->inst[inst];
    return mwg::Status::Ok();
}
} // namespace

extern "C" {

int32_t mw_abi_version(void) { return MW_ABI_VERSION; }

const char *mw_last_error(void) { return g_last_error.c_str(); }

mw_status mw_grid_plan(mw_plan *out, const mw_instance *inst, int32_t ninst, const mw_tuning *tuning,
                       void *stream) {
    try {
        if (!out) return fail(MW_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!inst || ninst < 1) return fail(MW_ERR_INVALID_ARG, "inst is NULL or ninst < 1");
        for (int i = 0; i < ninst; i++) {
            mwg::Status s = validate_instance(inst[i], i);
            if (!s.ok()) return fail(s);
        }
        if (tuning) {
            mwg::Status s = validate_tuning(*tuning);
            if (!s.ok()) return fail(s);
        }
        hipStream_t st = (hipStream_t)stream;
        size_t tmp_hint = 0;  // the largest instance's build in one temporary block
        for (int i = 0; i < ninst; i++)
            tmp_hint = std::max(tmp_hint, mwg::plan_tmp_hint(inst[i].nrow * (int64_t)inst[i].nchan, inst[i].nx, inst[i].ny));
        mwg::TmpScope scratch(st, tmp_hint);  // the build's temporaries, freed after the last sync below
        mwg::Plan *P = new mwg::Plan();
        if (hipGetDevice(&P->device) != hipSuccess) {
            delete P;
            return fail(MW_ERR_HIP, "hipGetDevice failed (no GPU?)");
        }
        // a plan of several instances settles its tile size across them before sorting any
        const bool autotune = tuning && tuning->autotune;
        const bool defer = ninst > 1 && !autotune;
        for (int i = 0; i < ninst; i++) P->inst.push_back(new mwg::Instance());
        {
            // instances are independent: plans of several are built by parallel host threads
            auto build = [&](int i, hipStream_t s) {
                return mwg::build_instance(*P->inst[i], inst[i], tuning, s, !defer, ninst > 1);
            };
            mwg::Status s;
            if (ninst >= kParallelPlan) {
                s = mwg::parallel_instances(P->device, ninst, st, build, tmp_hint);
            } else {
                for (int i = 0; i < ninst && s.ok(); i++) s = build(i, st);
            }
            if (!s.ok()) {
                destroy_plan(P);
                return fail(s);
            }
        }
        {
            // the tuner forms (and times) the batch itself; otherwise form it here
            mwg::Status s = autotune ? mwg::autotune_plan(*P, *tuning, st)
                            : ninst > 1                  ? mwg::batch_prepare(*P, st)
                                                         : mwg::Status::Ok();
            if (!s.ok()) {
                destroy_plan(P);
                return fail(s);
            }
        }
        if (hipStreamSynchronize(st) != hipSuccess) {
            destroy_plan(P);
            return fail(MW_ERR_HIP, "hipStreamSynchronize failed after planning");
        }
        {
            std::lock_guard<std::mutex> lk(g_plans_mu);
            g_plans.insert((void *)P);
        }
        *out = (mw_plan)P;
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(MW_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_grid_plan");
    }
}

mw_status mw_grid(mw_plan plan, const void *const *vis, const void *const *gains, void *const *grid,
                  int32_t accumulate, void *stream) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        if (!vis || !grid) return fail(MW_ERR_INVALID_ARG, "vis and grid arrays are required");
        mwg::Plan *P = (mwg::Plan *)plan;
        const int n = (int)P->inst.size();
        for (int i = 0; i < n; i++) {
            if (!grid[i] || (!vis[i] && P->inst[i]->ngroups > 0))
                return fail(MW_ERR_INVALID_ARG, "vis[i] and grid[i] must be device pointers");
            const uintptr_t align = P->inst[i]->npol >= 2 ? 16 : 8;
            if (((uintptr_t)vis[i] % align) || ((uintptr_t)grid[i] % 8))
                return fail(MW_ERR_INVALID_ARG, "vis must be 16-byte aligned (8 for npol 1), grid 8-byte");
            if (gains && gains[i] && !P->inst[i]->has_ants)
                return fail(MW_ERR_STATE, "gains given for an instance planned without antennas");
        }
        hipStream_t st = (hipStream_t)stream;
        if (n > 1 && P->batch) {
            s = mwg::batch_grid(*P, vis, gains, grid, accumulate ? 1 : 0, st);
            if (!s.ok()) return fail(s);
            return ok();
        }
        for (int i = 0; i < n; i++) {
            s = mwg::launch_grid(*P->inst[i], (const float2 *)vis[i],
                                 gains ? (const float2 *)gains[i] : nullptr, (float2 *)grid[i],
                                 accumulate ? 1 : 0, st);
            if (!s.ok()) return fail(s);
        }
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_grid");
    }
}

mw_status mw_grid_noalloc(mw_plan plan, const void *const *vis, const void *const *gains, void *const *grid,
                          int32_t accumulate, void *stream) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        if (!vis || !grid) return fail(MW_ERR_INVALID_ARG, "vis and grid arrays are required");
        mwg::Plan *P = (mwg::Plan *)plan;
        const int n = (int)P->inst.size();
        for (int i = 0; i < n; i++) {
            if (!grid[i] || (!vis[i] && P->inst[i]->ngroups > 0))
                return fail(MW_ERR_INVALID_ARG, "vis[i] and grid[i] must be device pointers");
            const uintptr_t align = P->inst[i]->npol >= 2 ? 16 : 8;
            if (((uintptr_t)vis[i] % align) || ((uintptr_t)grid[i] % 8))
                return fail(MW_ERR_INVALID_ARG, "vis must be 16-byte aligned (8 for npol 1), grid 8-byte");
            if (gains && gains[i] && !P->inst[i]->has_ants)
                return fail(MW_ERR_STATE, "gains given for an instance planned without antennas");
        }
        void *scr = nullptr;
        size_t cap = 0;
        s = mwg::static_scratch(&scr, &cap);
        if (!s.ok()) return fail(s);
        // instance by instance in stream order (a batched plan too: its graph is not used), each
        // reusing the whole scratch array
        for (int i = 0; i < n; i++) {
            s = mwg::launch_grid_into(*P->inst[i], (const float2 *)vis[i], gains ? (const float2 *)gains[i] : nullptr,
                                      (float2 *)grid[i], accumulate ? 1 : 0, (float *)scr, cap, (hipStream_t)stream);
            if (!s.ok()) return fail(s);
        }
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_grid_noalloc");
    }
}

mw_status mw_degrid(mw_plan plan, const void *const *grid, const void *const *gains,
                    const void *const *vis_in, void *const *vis_out, void *const *grad_gains, void *stream) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        if (!grid || !vis_out) return fail(MW_ERR_INVALID_ARG, "grid and vis_out arrays are required");
        mwg::Plan *P = (mwg::Plan *)plan;
        const int n = (int)P->inst.size();
        for (int i = 0; i < n; i++) {
            mwg::Instance &I = *P->inst[i];
            if (!grid[i] || (!vis_out[i] && I.ngroups > 0))
                return fail(MW_ERR_INVALID_ARG, "grid[i] and vis_out[i] must be device pointers");
            const bool g = gains && gains[i];
            const bool gg = grad_gains && grad_gains[i];
            if ((g || gg) && !I.has_ants)
                return fail(MW_ERR_STATE, "gains or grad_gains for an instance planned without antennas");
            if (gg && (!g || !vis_in || !vis_in[i]))
                return fail(MW_ERR_INVALID_ARG, "grad_gains needs gains and vis_in");
            const uintptr_t align = I.npol >= 2 ? 16 : 8;
            if (((uintptr_t)vis_out[i] % align) || (vis_in && ((uintptr_t)vis_in[i] % align)))
                return fail(mwg::make_error(MW_ERR_INVALID_ARG, "vis_out[i] and vis_in[i] must be %d-byte aligned",
                                            (int)align));
        }
        hipStream_t st = (hipStream_t)stream;
        if (n > 1 && P->batch) {
            s = mwg::batch_degrid(*P, grid, gains, vis_in, vis_out, grad_gains, st);
            if (!s.ok()) return fail(s);
            return ok();
        }
        for (int i = 0; i < n; i++) {
            s = mwg::launch_degrid(*P->inst[i], (const float2 *)grid[i],
                                   gains ? (const float2 *)gains[i] : nullptr,
                                   vis_in ? (const float2 *)vis_in[i] : nullptr, (float2 *)vis_out[i],
                                   grad_gains ? (float2 *)grad_gains[i] : nullptr, st);
            if (!s.ok()) return fail(s);
        }
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_degrid");
    }
}

mw_status mw_image(mw_plan plan, const void *const *in, void *const *out, int32_t direction,
                   int32_t correct, void *stream) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        if (!in || !out) return fail(MW_ERR_INVALID_ARG, "in and out arrays are required");
        if (direction != 1 && direction != -1) return fail(MW_ERR_INVALID_ARG, "direction must be +1 or -1");
        mwg::Plan *P = (mwg::Plan *)plan;
        for (size_t i = 0; i < P->inst.size(); i++) {
            if (!in[i] || !out[i]) return fail(MW_ERR_INVALID_ARG, "in[i] and out[i] must be device pointers");
            if (correct && P->inst[i]->stacks)
                return fail(MW_ERR_STATE, "correction is defined for the built-in kernel only");
        }
        for (size_t i = 0; i < P->inst.size(); i++) {
            s = mwg::launch_image(*P->inst[i], (const float2 *)in[i], (float2 *)out[i], direction,
                                  correct ? 1 : 0, (hipStream_t)stream);
            if (!s.ok()) return fail(s);
        }
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_image");
    }
}

mw_status mw_stokes(mw_plan plan, const void *const *images, const void *const *jones, void *const *out,
                    void *stream) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        if (!images || !out) return fail(MW_ERR_INVALID_ARG, "images and out arrays are required");
        mwg::Plan *P = (mwg::Plan *)plan;
        for (size_t i = 0; i < P->inst.size(); i++) {
            if (!images[i] || !out[i]) return fail(MW_ERR_INVALID_ARG, "images[i] and out[i] must be device pointers");
            if (P->inst[i]->npol != 4) return fail(MW_ERR_STATE, "Stokes conversion needs 4 polarisations");
        }
        for (size_t i = 0; i < P->inst.size(); i++) {
            s = mwg::launch_stokes(*P->inst[i], (const float2 *)images[i],
                                   jones ? (const float2 *)jones[i] : nullptr, (float *)out[i],
                                   (hipStream_t)stream);
            if (!s.ok()) return fail(s);
        }
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_stokes");
    }
}

mw_status mw_predict(mw_plan plan, int32_t inst, const double *sources, int32_t nsrc, const void *gains, void *vis,
                     int32_t accumulate, void *stream) {
    try {
        mwg::Instance *I = nullptr;
        mwg::Status s = check_inst(plan, inst, &I);
        if (!s.ok()) return fail(s);
        if ((!vis && I->ngroups > 0) || (!sources && nsrc > 0))
            return fail(MW_ERR_INVALID_ARG, "vis and sources must be device pointers");
        s = mwg::launch_predict(*I, sources, nsrc, (const float2 *)gains, (float2 *)vis, accumulate ? 1 : 0,
                                (hipStream_t)stream);
        return s.ok() ? ok() : fail(s);
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_predict");
    }
}

mw_status mw_solve_gains(mw_plan plan, int32_t inst, const void *vis, const void *model, const float *weights,
                         void *gains, int32_t niter, float *rel_step, void *stream) {
    try {
        mwg::Instance *I = nullptr;
        mwg::Status s = check_inst(plan, inst, &I);
        if (!s.ok()) return fail(s);
        if (!I->has_ants) return fail(MW_ERR_STATE, "gain solving needs an instance planned with antennas");
        if (!gains || ((!vis || !model) && I->ngroups > 0))
            return fail(MW_ERR_INVALID_ARG, "vis, model and gains must be device pointers");
        const uintptr_t align = I->npol >= 2 ? 16 : 8;
        if (((uintptr_t)vis % align) || ((uintptr_t)model % align) || ((uintptr_t)gains % 8))
            return fail(mwg::make_error(MW_ERR_INVALID_ARG, "vis and model must be %d-byte aligned, gains 8-byte",
                                        (int)align));
        s = mwg::launch_solve_gains(*I, (const float2 *)vis, (const float2 *)model, weights, (float2 *)gains, niter,
                                    rel_step, (hipStream_t)stream);
        return s.ok() ? ok() : fail(s);
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_solve_gains");
    }
}

mw_status mw_peel(mw_plan plan, int32_t inst, const void *vis, const double *sources, int32_t nsrc,
                  const float *weights, int32_t niter, void *resid, void *gains, float *rel_step, void *stream) {
    try {
        mwg::Instance *I = nullptr;
        mwg::Status s = check_inst(plan, inst, &I);
        if (!s.ok()) return fail(s);
        if (!I->has_ants) return fail(MW_ERR_STATE, "peeling needs an instance planned with antennas");
        if (((!vis || !resid) && I->ngroups > 0) || (nsrc > 0 && (!sources || !gains)))
            return fail(MW_ERR_INVALID_ARG, "vis, resid, gains (device) and sources (host) are required");
        const uintptr_t align = I->npol >= 2 ? 16 : 8;
        if (((uintptr_t)vis % align) || ((uintptr_t)resid % align) || ((uintptr_t)gains % 8))
            return fail(mwg::make_error(MW_ERR_INVALID_ARG, "vis and resid must be %d-byte aligned, gains 8-byte",
                                        (int)align));
        s = mwg::launch_peel(*I, (const float2 *)vis, sources, nsrc, weights, niter, (float2 *)resid, (float2 *)gains,
                             rel_step, (hipStream_t)stream);
        return s.ok() ? ok() : fail(s);
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_peel");
    }
}

mw_status mw_wstack_combine(mw_plan plan, const void *const *images, void *out, int32_t accumulate, void *stream) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        mwg::Plan *P = (mwg::Plan *)plan;
        if (!images || !out) return fail(MW_ERR_INVALID_ARG, "images and out are required");
        for (size_t i = 0; i < P->inst.size(); i++)
            if (!images[i]) return fail(MW_ERR_INVALID_ARG, "images[i] must be device pointers");
        s = mwg::launch_wstack_combine(*P, images, (float2 *)out, accumulate ? 1 : 0, (hipStream_t)stream);
        return s.ok() ? ok() : fail(s);
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_wstack_combine");
    }
}

mw_status mw_plan_info(mw_plan plan, int32_t inst, mw_plan_stats *out) {
    try {
        if (!plan || !out) return fail(MW_ERR_INVALID_ARG, "plan and out are required");
        if (!plan_is_live(plan)) return fail(MW_ERR_STATE, "plan is not live (destroyed?)");
        mwg::Plan *P = (mwg::Plan *)plan;
        if (inst < -1 || inst >= (int)P->inst.size()) return fail(MW_ERR_INVALID_ARG, "inst out of range");
        std::memset(out, 0, sizeof *out);
        for (int i = 0; i < (int)P->inst.size(); i++) {
            if (inst >= 0 && i != inst) continue;
            const mwg::Instance &I = *P->inst[i];
            out->ngroups += I.ngroups;
            out->nkept += I.nkept;
            out->nflagged += I.nflagged;
            out->noutside += I.noutside;
            out->ntiles += I.ntiles_nonempty;
            out->nwork += I.nwork;
            out->plan_bytes += I.arena.bytes;
            out->tile = I.L.tile;
            out->split = I.L.split;
            out->wg_waves = I.L.wg_waves;
            out->order = I.L.order;
            out->variant = I.L.variant;
            out->flush = I.L.flush;
            out->schedule = I.L.schedule;
        }
        out->batched = P->batch ? 1 : 0;
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_plan_info");
    }
}

mw_status mw_plan_order(mw_plan plan, int32_t inst, uint32_t *order_host) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        mwg::Plan *P = (mwg::Plan *)plan;
        if (inst < 0 || inst >= (int)P->inst.size() || !order_host)
            return fail(MW_ERR_INVALID_ARG, "inst out of range or order_host NULL");
        const mwg::Instance &I = *P->inst[inst];
        if (I.nkept > 0 && hipMemcpy(order_host, I.perm, 4 * (size_t)I.nkept, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(MW_ERR_HIP, "hipMemcpy of the gridding order failed");
        return MW_OK;
    } catch (const std::bad_alloc &) {
        return fail(MW_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception");
    }
}

mw_status mw_plan_positions(mw_plan plan, int32_t inst, int32_t *pos_host) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        mwg::Plan *P = (mwg::Plan *)plan;
        if (inst < 0 || inst >= (int)P->inst.size() || !pos_host)
            return fail(MW_ERR_INVALID_ARG, "inst out of range or pos_host NULL");
        const mwg::Instance &I = *P->inst[inst];
        std::vector<uint32_t> packed((size_t)I.ngroups);
        if (I.ngroups > 0 &&
            hipMemcpy(packed.data(), I.pos, 4 * (size_t)I.ngroups, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(MW_ERR_HIP, "hipMemcpy of positions failed");
        const int half = I.O / 2;
        for (int64_t g = 0; g < I.ngroups; g++) {
            const uint32_t p = packed[g];
            int32_t *o = pos_host + 4 * g;
            if (p == mwg::kDropped) {
                o[0] = o[1] = o[2] = o[3] = -1;
            } else {
                o[0] = (int32_t)(p & 0xFFFu);
                o[1] = (int32_t)((p >> 12) & 0xFFFu);
                o[2] = (int32_t)((p >> 24) & 0xFu) - half;
                o[3] = (int32_t)(p >> 28) - half;
            }
        }
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_plan_positions");
    }
}

mw_status mw_plan_tables(mw_plan plan, int32_t inst, float *table_host, float *corr_x, float *corr_y) {
    try {
        if (!plan) return fail(MW_ERR_INVALID_ARG, "plan is NULL");
        if (!plan_is_live(plan)) return fail(MW_ERR_STATE, "plan is not live (destroyed?)");
        mwg::Plan *P = (mwg::Plan *)plan;
        if (inst < 0 || inst >= (int)P->inst.size()) return fail(MW_ERR_INVALID_ARG, "inst out of range");
        const mwg::Instance &I = *P->inst[inst];
        if (I.stacks) return fail(MW_ERR_STATE, "instance uses kernel stacks");
        if (table_host) std::memcpy(table_host, I.h_tab.data(), 4 * I.h_tab.size());
        if (corr_x) std::memcpy(corr_x, I.h_corrx.data(), 4 * I.h_corrx.size());
        if (corr_y) std::memcpy(corr_y, I.h_corry.data(), 4 * I.h_corry.size());
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_plan_tables");
    }
}

mw_status mw_plan_set_timing(mw_plan plan, int32_t enable) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        mwg::Plan *P = (mwg::Plan *)plan;
        for (mwg::Instance *I : P->inst) {
            if (enable)
                for (hipEvent_t &e : I->tev)
                    if (!e && hipEventCreate(&e) != hipSuccess) return fail(MW_ERR_HIP, "hipEventCreate failed");
            I->timing = enable != 0;
            I->timed = false;
        }
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_plan_set_timing");
    }
}

mw_status mw_plan_kernel_ms(mw_plan plan, int32_t inst, float *grid_ms, float *merge_ms) {
    try {
        mwg::Status s = check_plan(plan);
        if (!s.ok()) return fail(s);
        mwg::Plan *P = (mwg::Plan *)plan;
        if (inst < 0 || inst >= (int)P->inst.size()) return fail(MW_ERR_INVALID_ARG, "inst out of range");
        mwg::Instance &I = *P->inst[inst];
        if (!I.timed) return fail(MW_ERR_STATE, "no timed mw_grid call on this instance");
        if (hipEventSynchronize(I.tev[2]) != hipSuccess) return fail(MW_ERR_HIP, "hipEventSynchronize failed");
        float g = 0.f, m = 0.f;
        if (hipEventElapsedTime(&g, I.tev[0], I.tev[1]) != hipSuccess ||
            hipEventElapsedTime(&m, I.tev[1], I.tev[2]) != hipSuccess)
            return fail(MW_ERR_HIP, "hipEventElapsedTime failed");
        if (grid_ms) *grid_ms = g;
        if (merge_ms) *merge_ms = m;
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_plan_kernel_ms");
    }
}

mw_status mw_plan_destroy(mw_plan plan) {
    try {
        if (!plan) return ok();
        {
            std::lock_guard<std::mutex> lk(g_plans_mu);
            if (!g_plans.erase((void *)plan)) return fail(MW_ERR_STATE, "plan is not live (destroyed twice?)");
        }
        destroy_plan((mwg::Plan *)plan);
        return ok();
    } catch (...) {
        return fail(MW_ERR_HIP, "unexpected exception in mw_plan_destroy");
    }
}

} // extern "C"
