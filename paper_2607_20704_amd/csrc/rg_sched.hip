// rg_sched.hip -- kernel schedule of a tree and the scheduled level update.
//
// Paper Sec. 3: grouping octs into larger blocks (nsubgrid) shares the
// stencil and removes redundant ghost-cell work; in a cell-by-cell tree only
// some regions are covered by complete blocks.  The schedule finds, per
// level, the complete Hilbert-aligned 8^3-oct bricks that border no coarse
// ghost, then among the other octs the complete sibling groups (8 octs of
// one father, consecutive keys), and lists the remaining octs for the
// per-oct kernel.
#include <vector>

#include "rg_internal.hpp"

namespace rg {
rg_status hydro_level_list(const double *uold, double *unew, const int32_t *nbr27, const uint32_t *son,
                           const int32_t *list, int64_t count, double *corr, int64_t corr_base, const double *dt,
                           double dx, double gamma, int form, const rg_tuning *tune, double cfl, double *dt_next,
                           hipStream_t s, int64_t first = 0, const double *ucoarse = nullptr,
                           int corr_mode = 0, int ghost = 0, const double *ucoarse2 = nullptr);
rg_status hydro_groups_list(const double *uold, double *unew, const int32_t *nbr27, const uint32_t *son,
                            const int32_t *father, const int32_t *list, int64_t count, double *corr,
                            int64_t corr_base, const double *dt, double dx, double gamma, int form,
                            const rg_tuning *tune, double cfl, double *dt_next, hipStream_t s, const double *ucoarse,
                            int corr_mode, int ghost, const double *ucoarse2);
rg_status hydro_bricks(const double *uold, double *unew, const int32_t *nbr27, const uint32_t *son,
                       const uint64_t *keys, const int32_t *bricks, int64_t nbricks, const double *dt, double dx,
                       double gamma, int outflow, int form, double cfl, double *dt_next, int waves, hipStream_t s,
                       int64_t pair_first, int pair_level);
}  // namespace rg

using namespace rg;

namespace {
constexpr int64_t kBrickOcts = 512;
constexpr int64_t kGroupOcts = 8;
// neighbour-list slots (dx+1) + 3 (dy+1) + 9 (dz+1) of the faces x-, x+, y-, y+, z-, z+
constexpr int kFaceSlot[6] = {12, 14, 10, 16, 4, 22};
}

namespace rg {

// One level of tree t: with a schedule, its bricks by the brick kernel, its
// complete sibling groups by the group kernel and the rest by the per-oct
// kernel; without one, the whole level by the per-oct kernel.  Coarse ghost
// cells are read from ucoarse (bricks have none).  The fluxes owed to coarse
// cells go to corr (30 doubles per oct from the first oct above lmin):
// stored (corr_mode 0), stored as 0 + flux (1) or added (2).
rg_status hydro_tree_level(const rg_tree *t, const rg_schedule *sc, int level, const double *d_dt, double gamma,
                           const double *d_uold, const double *d_ucoarse, double *d_unew, double cfl,
                           double *d_dt_next, int form, const rg_tuning *tune, hipStream_t s, double *d_corr,
                           int corr_mode, const double *d_ucoarse2)
{
    RG_REQUIRE(t->ghost == RG_GHOST_INJECT || t->ghost == RG_GHOST_LINEAR, "bad ghost mode %d", t->ghost);
    const double dx = ldexp(1.0, -level);
    const int64_t corr_base = t->level_begin[t->lmin + 1];
    double *corr = level > t->lmin ? d_corr : nullptr;
    const bool bricks = sc && !(tune && tune->no_bricks);
    if (bricks) {
        // a complete periodic level without split cells (the finest, with
        // every oct in a brick): its bricks go two by two along z
        const int64_t nl = t->level_begin[level + 1] - t->level_begin[level];
        const bool pairs = !(tune && tune->no_pairs) && level >= 5 && level == t->lmax &&
                           t->bc == RG_BC_PERIODIC && nl == (int64_t(1) << (3 * (level - 1))) &&
                           sc->brick_count[level] * 512 == nl;
        RG_TRY(hydro_bricks(d_uold, d_unew, t->d_nbr27, t->d_son_mask, t->d_keys, sc->d_list + sc->brick_begin[level],
                            sc->brick_count[level], d_dt, dx, gamma, t->bc == RG_BC_OUTFLOW, form, cfl, d_dt_next,
                            tune ? tune->brick_waves : 0, s, t->level_begin[level], pairs ? level : -1));
        if (tune && tune->no_groups) {
            RG_TRY(hydro_level_list(d_uold, d_unew, t->d_nbr27, t->d_son_mask, sc->d_list + sc->rest_begin[level],
                                    sc->rest_count[level], corr, corr_base, d_dt, dx, gamma, form, tune, cfl,
                                    d_dt_next, s, 0, d_ucoarse, corr_mode, t->ghost, d_ucoarse2));
        } else {
            RG_TRY(hydro_groups_list(d_uold, d_unew, t->d_nbr27, t->d_son_mask, t->d_father_cell,
                                     sc->d_list + sc->group_begin[level], sc->group_count[level], corr, corr_base,
                                     d_dt, dx, gamma, form, tune, cfl, d_dt_next, s, d_ucoarse, corr_mode, t->ghost,
                                     d_ucoarse2));
            RG_TRY(hydro_level_list(d_uold, d_unew, t->d_nbr27, t->d_son_mask, sc->d_list + sc->single_begin[level],
                                    sc->single_count[level], corr, corr_base, d_dt, dx, gamma, form, tune, cfl,
                                    d_dt_next, s, 0, d_ucoarse, corr_mode, t->ghost, d_ucoarse2));
        }
    } else {
        RG_TRY(hydro_level_list(d_uold, d_unew, t->d_nbr27, t->d_son_mask, nullptr,
                                t->level_begin[level + 1] - t->level_begin[level], corr, corr_base, d_dt, dx, gamma,
                                form, tune, cfl, d_dt_next, s, t->level_begin[level], d_ucoarse, corr_mode, t->ghost,
                                d_ucoarse2));
    }
    return RG_OK;
}

}  // namespace rg

extern "C" {

rg_status rg_schedule_build(const rg_tree *t, int32_t *d_list, int64_t capacity, rg_schedule *out, void *stream)
{
    RG_REQUIRE(t && d_list && out, "null pointer");
    RG_REQUIRE(t->n_oct > 0 && capacity >= 4 * t->n_oct, "list capacity below 4 n_oct");
    RG_REQUIRE(t->lmin >= 1 && t->lmax >= t->lmin && t->lmax <= RG_MAX_LEVEL, "bad levels");
    const int64_t n = t->n_oct;
    hipStream_t s = as_stream(stream);
    std::vector<uint64_t> keys(n);
    std::vector<int32_t> nbr(static_cast<size_t>(27) * n);
    hipError_t e = hipMemcpyAsync(keys.data(), t->d_keys, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(nbr.data(), t->d_nbr27, nbr.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(RG_EHIP, "schedule readback: %s", hipGetErrorString(e));

    std::vector<int32_t> list, all_bricks, other;
    std::vector<std::vector<int32_t>> groups(RG_MAX_LEVEL + 2), singles(RG_MAX_LEVEL + 2);
    list.reserve(2 * n);
    for (int l = 0; l < RG_MAX_LEVEL + 2; ++l)
        out->brick_begin[l] = out->brick_count[l] = out->rest_begin[l] = out->rest_count[l] = out->border_begin[l] =
            out->border_count[l] = out->group_begin[l] = out->group_count[l] = out->single_begin[l] =
                out->single_count[l] = 0;
    for (int l = t->lmin; l <= t->lmax; ++l) {
        const int64_t b = t->level_begin[l], end = t->level_begin[l + 1];
        std::vector<uint8_t> covered(end - b, 0), complete(end - b, 0);
        out->brick_begin[l] = static_cast<int64_t>(list.size());
        for (int64_t o = b; o + kBrickOcts <= end;) {
            const uint64_t k = keys[o];
            if ((k & (kBrickOcts - 1)) == 0 && keys[o + kBrickOcts - 1] == k + kBrickOcts - 1) {
                all_bricks.push_back(static_cast<int32_t>(o));
                for (int64_t q = o; q < o + kBrickOcts; ++q) complete[q - b] = 1;
                bool coarse = false;
                for (int64_t q = o; q < o + kBrickOcts && !coarse; ++q)
                    for (int j = 0; j < 27; ++j) {
                        const int32_t v = nbr[27 * q + j];
                        if (v < 0 && v != RG_NBR_OUTSIDE) { coarse = true; break; }
                    }
                if (!coarse) {
                    list.push_back(static_cast<int32_t>(o));
                    for (int64_t q = o; q < o + kBrickOcts; ++q) covered[q - b] = 1;
                }
                o += kBrickOcts;
            } else {
                ++o;
            }
        }
        out->brick_count[l] = static_cast<int64_t>(list.size()) - out->brick_begin[l];
        out->rest_begin[l] = static_cast<int64_t>(list.size());
        for (int64_t o = b; o < end; ++o)
            if (!covered[o - b]) list.push_back(static_cast<int32_t>(o));
        out->rest_count[l] = static_cast<int64_t>(list.size()) - out->rest_begin[l];
        for (int64_t o = b; o < end; ++o)
            if (!complete[o - b]) other.push_back(static_cast<int32_t>(o));
        // complete sibling groups outside the bricks (a brick holds whole
        // groups); their father cells exist above lmin only
        std::vector<uint8_t> grouped(end - b, 0);
        if (l > t->lmin)
            for (int64_t o = b; o + kGroupOcts <= end; ++o) {
                const uint64_t k = keys[o];
                if (!covered[o - b] && (k & (kGroupOcts - 1)) == 0 && keys[o + kGroupOcts - 1] == k + kGroupOcts - 1) {
                    groups[l].push_back(static_cast<int32_t>(o));
                    for (int64_t q = o; q < o + kGroupOcts; ++q) grouped[q - b] = 1;
                }
            }
        for (int64_t o = b; o < end; ++o)
            if (!covered[o - b] && !grouped[o - b]) singles[l].push_back(static_cast<int32_t>(o));
    }
    out->nbr_brick_begin = static_cast<int64_t>(list.size());
    out->nbr_brick_count = static_cast<int64_t>(all_bricks.size());
    list.insert(list.end(), all_bricks.begin(), all_bricks.end());
    out->nbr_rest_begin = static_cast<int64_t>(list.size());
    out->nbr_rest_count = static_cast<int64_t>(other.size());
    list.insert(list.end(), other.begin(), other.end());
    // octs above lmin with a coarse cell across a face, level by level
    for (int l = t->lmin + 1; l <= t->lmax; ++l) {
        out->border_begin[l] = static_cast<int64_t>(list.size());
        for (int64_t o = t->level_begin[l]; o < t->level_begin[l + 1]; ++o) {
            bool coarse = false;
            for (int side = 0; side < 6; ++side) {
                const int32_t v = nbr[27 * o + kFaceSlot[side]];
                coarse = coarse || (v < 0 && v != RG_NBR_OUTSIDE);
            }
            if (coarse) list.push_back(static_cast<int32_t>(o));
        }
        out->border_count[l] = static_cast<int64_t>(list.size()) - out->border_begin[l];
    }
    for (int l = t->lmin; l <= t->lmax; ++l) {
        out->group_begin[l] = static_cast<int64_t>(list.size());
        out->group_count[l] = static_cast<int64_t>(groups[l].size());
        list.insert(list.end(), groups[l].begin(), groups[l].end());
    }
    for (int l = t->lmin; l <= t->lmax; ++l) {
        out->single_begin[l] = static_cast<int64_t>(list.size());
        out->single_count[l] = static_cast<int64_t>(singles[l].size());
        list.insert(list.end(), singles[l].begin(), singles[l].end());
    }
    if (static_cast<int64_t>(list.size()) > capacity) return fail(RG_EINVAL, "schedule exceeds list capacity");
    if (!list.empty()) {
        e = hipMemcpyAsync(d_list, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(RG_EHIP, "schedule upload: %s", hipGetErrorString(e));
    }
    out->d_list = d_list;
    return RG_OK;
}

rg_status rg_hydro_step_scheduled(const rg_tree *t, const rg_schedule *sc, int level, const double *d_dt,
                                  double gamma, const double *d_uold, double *d_unew, double cfl, double *d_dt_next,
                                  int form, const rg_tuning *tune, void *stream)
{
    RG_REQUIRE(t && sc && sc->d_list && d_dt && d_uold && d_unew, "null pointer");
    RG_REQUIRE(level >= t->lmin && level <= t->lmax, "level %d not in the tree", level);
    RG_REQUIRE(d_uold != d_unew, "uold and unew must not alias");
    RG_REQUIRE(form == RG_FP64 || form == RG_MIXED, "bad form %d", form);
    RG_REQUIRE(gamma > 1, "bad gamma");
    RG_REQUIRE(!d_dt_next || (cfl > 0 && aligned(d_dt_next, 8)), "bad cfl or misaligned dt_next");
    return hydro_tree_level(t, sc, level, d_dt, gamma, d_uold, d_uold, d_unew, cfl, d_dt_next, form, tune,
                            as_stream(stream), t->d_corr, 0, d_uold);
}

}  // extern "C"
