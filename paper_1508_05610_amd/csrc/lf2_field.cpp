// lf2_field.cpp -- C ABI of the field operations (lf2_kfield.hip).
#include <stdint.h>

#include <cmath>

#include "lf2_internal.hpp"
#include "lf2_plan.hpp"

using namespace lf2;
using namespace lf2::host;

namespace {

lf2_status check_lattice(const lf2_lattice *lat, int32_t ncomp, int64_t n[3])
{
    if (!lat) return fail(LF2_ERR_INVALID_ARG, "lattice is NULL");
    if (lat->dim != 3) return fail(LF2_ERR_UNSUPPORTED, "dim %d: field operations are 3-d", lat->dim);
    if (lat->halo < 0) return fail(LF2_ERR_INVALID_ARG, "halo %d < 0", lat->halo);
    if (ncomp < 1 || ncomp > 64) return fail(LF2_ERR_INVALID_ARG, "ncomp %d outside [1, 64]", ncomp);
    for (int i = 0; i < 3; ++i) {
        if (lat->size[i] < 1) return fail(LF2_ERR_INVALID_ARG, "size[%d] < 1", i);
        n[i] = lat->size[i];
    }
    return LF2_OK;
}

}  // namespace

extern "C" {

lf2_status lf2_update_halo(const lf2_lattice *lat, int32_t ncomp, int32_t elem_bytes, void *field,
                           void *stream)
{
    int64_t n[3];
    lf2_status st;
    if ((st = check_lattice(lat, ncomp, n))) return st;
    if (elem_bytes != 4 && elem_bytes != 8)
        return fail(LF2_ERR_UNSUPPORTED, "elem_bytes %d: 4 (float) or 8 (complex float)", elem_bytes);
    if ((st = check_ptr(field, "field", 4))) return st;
    if (lat->halo > lat->size[0] || lat->halo > lat->size[1] || lat->halo > lat->size[2])
        return fail(LF2_ERR_UNSUPPORTED, "halo %d wider than the lattice", lat->halo);
    LF2_HIP(launch_update_halo(field, n, lat->halo, (int64_t)ncomp * elem_bytes / 4,
                               (hipStream_t)stream));
    return LF2_OK;
}

lf2_status lf2_gradient(const lf2_lattice *lat, int32_t ncomp, const float *in, float *out,
                        double dx, void *stream)
{
    int64_t n[3];
    lf2_status st;
    if ((st = check_lattice(lat, ncomp, n))) return st;
    if (lat->halo < 1) return fail(LF2_ERR_INVALID_ARG, "the derivative reads neighbours: halo >= 1");
    if ((st = check_ptr(in, "in", 4)) || (st = check_ptr(out, "out", 4))) return st;
    if ((const void *)in == (const void *)out) return fail(LF2_ERR_INVALID_ARG, "in and out must not alias");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LF2_ERR_INVALID_ARG, "dx must be > 0");
    LF2_HIP(launch_gradient(in, out, n, lat->halo, ncomp, dx, (hipStream_t)stream));
    return LF2_OK;
}

}  // extern "C"
