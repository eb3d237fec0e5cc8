// rg_subcycle.hip -- one coarse step with level-by-level time steps.
//
// Paper Sec. 2: the hierarchy advances level by level with adaptive time
// steps, each level taking two steps of half its parent's.  The coarse step
// D is the CFL limit of every leaf scaled to the coarsest level; level l
// steps by D / 2^(l - lmin).  Advancing level l:
//   hydro of level l (own cells from its current state, coarse ghosts from
//   the coarser level's state at the start of that level's step);
//   twice { advance level l+1; acc += level l+1's coarse-side fluxes };
//   acc added to the coarse cells, side by side; level l+1 restricted into
//   level l's split cells.
//
// State buffers: every level lives in one of two buffers and flips to the
// other at each of its own steps, so nothing is copied between substeps.  A
// level above lmin takes an even number of steps per coarse step and ends in
// the buffer it started in; only level lmin ends in the other one and is
// copied back at the end.  The coarser level's old state stays untouched in
// its buffer while the finer level runs, because the coarser level's update
// writes the other buffer.
#include "rg_internal.hpp"

namespace rg {

rg_status hydro_tree_level(const rg_tree *t, const rg_schedule *sc, int level, const double *d_dt, double gamma,
                           const double *d_uold, const double *d_ucoarse, double *d_unew, double cfl,
                           double *d_dt_next, int form, const rg_tuning *tune, hipStream_t s, double *d_corr,
                           int corr_mode, const double *d_ucoarse2);
rg_status restrict_level2(const double *src, double *dst, const int32_t *father, int64_t ob, int64_t oe,
                          hipStream_t s);
rg_status coarse_corrections_list(double *unew, const double *corr, int64_t corr_base, const int32_t *nbr27,
                                  const int32_t *list, int64_t count, hipStream_t s);
rg_status cfl_dt_pass(const double *d_u, const uint32_t *d_son_mask, const int64_t *h_level_begin, int lmin, int lmax,
                      double gamma, double cfl, double *d_dt, int sub, void *stream);

namespace {

// dt[1 + k] = dt[0] / 2^k: the step of level lmin + k (exact halvings)
__global__ void k_level_dts(double *dt, int nlev)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (int k = 0; k < nlev; ++k) dt[1 + k] = ldexp(dt[0], -k);
}

struct Sub {
    const rg_tree *t;
    double *buf[2];
    int cur[RG_MAX_LEVEL + 2];   // buffer holding each level's current state
    double *acc;
    double *dt;                  // dt[1 + l - lmin]: level l's step
    double gamma;
    int form;
    const rg_tuning *tune;
    hipStream_t s;
};

// sub: which of its parent's two substeps this is (0 for lmin); the level's
// fluxes owed to coarse cells are summed over the two into acc
rg_status advance(Sub &c, int l, int sub)
{
    const rg_tree *t = c.t;
    const int64_t ob = t->level_begin[l], oe = t->level_begin[l + 1];
    const double *own = c.buf[c.cur[l]];
    double *out = c.buf[c.cur[l] ^ 1];
    const double *coarse = l > t->lmin ? c.buf[c.cur[l - 1]] : own;
    const double *coarse2 = l > t->lmin + 1 ? c.buf[c.cur[l - 2]] : coarse;
    if (oe > ob)
        RG_TRY(hydro_tree_level(t, t->sched, l, c.dt + 1 + (l - t->lmin), c.gamma, own, coarse, out, 0.0, nullptr,
                                c.form, c.tune, c.s, c.acc, 1 + sub, coarse2));
    if (l < t->lmax) {
        const int64_t fb = t->level_begin[l + 1], fe = t->level_begin[l + 2];
        const int64_t base = t->level_begin[t->lmin + 1];
        for (int s2 = 0; s2 < 2; ++s2) RG_TRY(advance(c, l + 1, s2));
        if (fe > fb) {
            if (t->sched) {
                const rg_schedule *sc = t->sched;
                RG_TRY(coarse_corrections_list(out, c.acc, base, t->d_nbr27, sc->d_list + sc->border_begin[l + 1],
                                               sc->border_count[l + 1], c.s));
            } else {
                RG_TRY(rg_apply_coarse_corrections(out, c.acc, base, t->d_nbr27, fb, fe, c.s));
            }
            RG_TRY(restrict_level2(c.buf[c.cur[l + 1]], out, t->d_father_cell, fb, fe, c.s));
        }
    }
    c.cur[l] ^= 1;
    return RG_OK;
}

}  // namespace
}  // namespace rg

using namespace rg;

extern "C" {

rg_status rg_step_subcycled(const rg_tree *t, double *d_u, double *d_scratch, double *d_acc, double gamma, double cfl,
                            int form, unsigned flags, double *d_dt, const rg_tuning *tune, void *stream)
{
    RG_REQUIRE(t && d_u && d_scratch && d_dt, "null pointer");
    RG_REQUIRE(t->n_oct > 0 && t->lmin >= 1 && t->lmax >= t->lmin && t->lmax <= RG_MAX_LEVEL, "bad tree");
    RG_REQUIRE(t->level_begin[t->lmin] == 0 && t->level_begin[t->lmax + 1] == t->n_oct, "bad level ranges");
    RG_REQUIRE(t->lmin == t->lmax || d_acc, "a multilevel tree needs an accumulation buffer");
    RG_REQUIRE((flags & ~(RG_STEP_REBUILD | RG_STEP_REKEY)) == 0, "unsupported flags %u", flags);
    RG_REQUIRE(d_u != d_scratch, "state and scratch must not alias");
    RG_REQUIRE(aligned(d_u, 8) && aligned(d_scratch, 8) && aligned(d_dt, 8) && (!d_acc || aligned(d_acc, 8)),
               "misaligned pointer");
    RG_REQUIRE(form == RG_FP64 || form == RG_MIXED, "bad form %d", form);
    RG_REQUIRE(gamma > 1 && cfl > 0, "bad gamma or cfl");
    hipStream_t s = as_stream(stream);
    const SinkScope sink(t->d_hash_ws);
    if (flags) RG_TRY(rg_prepare_tree(t, flags, stream));
    RG_TRY(cfl_dt_pass(d_u, t->d_son_mask, t->level_begin, t->lmin, t->lmax, gamma, cfl, d_dt, 1, stream));
    k_level_dts<<<1, 64, 0, s>>>(d_dt, t->lmax - t->lmin + 1);
    RG_TRY(launch_status("subcycle level steps"));
    Sub c;
    c.t = t;
    c.buf[0] = d_u;
    c.buf[1] = d_scratch;
    for (int l = 0; l < RG_MAX_LEVEL + 2; ++l) c.cur[l] = 0;
    c.acc = d_acc;
    c.dt = d_dt;
    c.gamma = gamma;
    c.form = form;
    c.tune = tune;
    c.s = s;
    RG_TRY(advance(c, t->lmin, 0));
    // level lmin took one step and sits in the scratch buffer; every finer
    // level took an even number and is back in d_u
    const int64_t nb = t->level_begin[t->lmin + 1] - t->level_begin[t->lmin];
    if (hipMemcpyAsync(d_u, d_scratch, static_cast<size_t>(nb) * 40 * sizeof(double), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return fail(RG_EHIP, "subcycle copy-back");
    return RG_OK;
}

}  // extern "C"
