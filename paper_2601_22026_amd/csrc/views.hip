// views.hip - training-view selection of the continual refinement (host code).
//
// The refinement keeps a set of training views and admits a new foveal view
// only when it is novel against every kept view: its centre lies farther than
// delta_pos from that view's centre, or the dot product of the two unit viewing
// directions is below cos(theta_view) (Method, "Periphery Model Training",
// Eq. (1); the paper uses delta_pos = 0.05 and theta_view = 5 degrees).  A few
// dozen views are compared per offer, so this runs on the host in double
// precision; it touches no device memory.
#include <cmath>
#include <new>

#include "gsfit.h"

namespace {

struct Pose {
    double c[3];
    double d[3];
};

// Centre and unit viewing direction (the camera's +z axis in world coordinates:
// the third row of the world-to-camera rotation).  False for a zero direction.
bool pose_of(const gsf_camera &cam, Pose *out) {
    double len2 = 0.0;
    for (int k = 0; k < 3; k++) {
        out->c[k] = (double)cam.campos[k];
        out->d[k] = (double)cam.viewmat[8 + k];
        len2 += out->d[k] * out->d[k];
    }
    const double len = std::sqrt(len2);
    if (!(len > 0.0) || !std::isfinite(len)) return false;
    for (int k = 0; k < 3; k++) out->d[k] /= len;
    for (int k = 0; k < 3; k++)
        if (!std::isfinite(out->c[k])) return false;
    return true;
}

bool novel(const Pose &q, const Pose &kept, double delta, double cos_t) {
    double d2 = 0.0, dot = 0.0;
    for (int k = 0; k < 3; k++) {
        const double e = q.c[k] - kept.c[k];
        d2 += e * e;
        dot += q.d[k] * kept.d[k];
    }
    return std::sqrt(d2) > delta || dot < cos_t;
}

}  // namespace

extern "C" gsf_status gsf_view_select(const gsf_camera *set, int32_t n_set, const gsf_camera *cand,
                                      int32_t n_cand, float delta_pos, float theta_view_deg,
                                      int32_t *keep, int32_t *n_kept) {
    if (n_set < 0 || n_cand < 0 || (n_set > 0 && !set) || (n_cand > 0 && (!cand || !keep)) ||
        !n_kept)
        return GSF_E_INVALID;
    if (!(delta_pos >= 0.f) || !std::isfinite(delta_pos) || !(theta_view_deg >= 0.f) ||
        !(theta_view_deg <= 180.f))
        return GSF_E_INVALID;
    const double delta = (double)delta_pos;
    const double cos_t = std::cos((double)theta_view_deg * (M_PI / 180.0));
    // the kept poses: the given set, then every accepted candidate
    Pose *poses = new (std::nothrow) Pose[(size_t)n_set + (size_t)n_cand + 1];
    if (!poses) return GSF_E_INVALID;
    int64_t np = 0;
    for (int32_t i = 0; i < n_set; i++) {
        if (!pose_of(set[i], &poses[np])) {
            delete[] poses;
            return GSF_E_INVALID;
        }
        np++;
    }
    // validate every candidate before writing any output
    for (int32_t j = 0; j < n_cand; j++) {
        Pose q;
        if (!pose_of(cand[j], &q)) {
            delete[] poses;
            return GSF_E_INVALID;
        }
    }
    int32_t kept = 0;
    for (int32_t j = 0; j < n_cand; j++) {
        Pose q;
        pose_of(cand[j], &q);
        bool ok = true;
        for (int64_t i = 0; i < np && ok; i++) ok = novel(q, poses[i], delta, cos_t);
        keep[j] = ok ? 1 : 0;
        if (ok) {
            poses[np++] = q;
            kept++;
        }
    }
    *n_kept = kept;
    delete[] poses;
    return GSF_OK;
}
