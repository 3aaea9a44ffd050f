// capi.hip -- the extern "C" boundary of libsph: host-side validation,
// workspace carving and the launch sequences of every entry point.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "sph_launch.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int check_hip(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SPH_EHIP, "%s: %s", what, hipGetErrorString(e));
    return SPH_OK;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int ceil_log2(int v)
{
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

}  // namespace

namespace sph {

constexpr double pi_d = 3.14159265358979323846;

// Default neighbour-table depth: 32 in 2D and 80 in 3D for Wendland C2; for
// the quintic spline 1.6 times the lattice count of the 3h ball plus 12, in
// multiples of 16 (80 in 2D and 336 in 3D at h = 1.2 dx).
static int32_t default_maxnb(const sph_params *prm)
{
    if (prm && (prm->flags & SPH_FLAG_QUINTIC) && prm->h > 0 && prm->dx > 0) {
        const double R = 3.0 * prm->h / prm->dx;
        const double ball = prm->dim == 3 ? 4.0 / 3.0 * pi_d * R * R * R : pi_d * R * R;
        const int m = int(std::ceil((1.6 * ball + 12.0) / 16.0)) * 16;
        return m < 32 ? 32 : (m > 1024 ? 1024 : m);
    }
    return prm && prm->dim == 3 ? 80 : 32;
}

// Validates the parameter block and derives the kernel constants.
static int make_dev(const sph_params *p, int64_t cap, int prec, int maxnb, Dev *k)
{
    if (!p) return fail(SPH_EINVAL, "params is NULL");
    if (p->dim == 1) return fail(SPH_EUNSUPPORTED, "dim 1 is not provided");
    if (p->dim != 2 && p->dim != 3) return fail(SPH_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->n_avg != kNavg) return fail(SPH_EINVAL, "n_avg must be %d (got %d)", kNavg, p->n_avg);
    {
        const double vals[] = {p->h, p->dx, p->rho0, p->c, p->U, p->nu, p->alpha, p->eta, p->dt,
                               p->pb, p->lo[0], p->lo[1], p->lo[2], p->hi[0], p->hi[1], p->hi[2],
                               p->x_inlet, p->x_outlet, p->x_outlet_end, p->inlet_len,
                               p->noise_amp};
        const char *names[] = {"h", "dx", "rho0", "c", "U", "nu", "alpha", "eta", "dt", "pb",
                               "lo[0]", "lo[1]", "lo[2]", "hi[0]", "hi[1]", "hi[2]", "x_inlet",
                               "x_outlet", "x_outlet_end", "inlet_len", "noise_amp"};
        for (size_t q = 0; q < sizeof vals / sizeof vals[0]; ++q)
            if (!std::isfinite(vals[q]))
                return fail(SPH_ENONFINITE, "parameter %s is not finite", names[q]);
    }
    if (!(p->h > 0) || !(p->dx > 0) || !(p->rho0 > 0) || !(p->c > 0) || !(p->dt > 0) ||
        !(p->eta > 0) || !(p->nu >= 0) || !(p->pb >= 0) || !(p->alpha >= 0) || !(p->U >= 0))
        return fail(SPH_EINVAL, "h, dx, rho0, c, dt, eta must be > 0 and nu, pb, alpha, U >= 0");
    if (p->dt * (p->c + p->U) > 0.5 * p->h)
        return fail(SPH_ECFL, "dt = %g exceeds the acoustic bound 0.5 h / (c + U) = %g", p->dt,
                    0.5 * p->h / (p->c + p->U));
    if (cap < 1 || cap > INT32_MAX) return fail(SPH_EINVAL, "cap must be in [1, 2^31)");
    if (p->list_cap < 0 || p->list_cap > 2048)
        return fail(SPH_EINVAL, "list_cap must be in [0, 2048] (got %d)", p->list_cap);
    if (p->outlet < SPH_OUTLET_HYBRID || p->outlet > SPH_OUTLET_MIRROR)
        return fail(SPH_EINVAL, "outlet must be an SPH_OUTLET_* rule (got %d)", p->outlet);
    if (prec != SPH_FP64 && prec != SPH_FP32) return fail(SPH_EINVAL, "bad precision %d", prec);
    std::memset(k, 0, sizeof *k);
    k->dim = p->dim;
    k->flags = p->flags;
    k->reuse = (p->flags & SPH_FLAG_REUSE_BINS) ? 1 : 0;
    k->outlet = p->outlet;
    k->quintic = (p->flags & SPH_FLAG_QUINTIC) ? 1 : 0;
    k->g_force = p->group_force;
    k->g_nbr = p->group_nbr;
    k->prec = prec;
    k->maxnb = maxnb;
    k->cap = cap;
    k->h = p->h;
    // the kernel's support: 2h (Wendland C2) or 3h (the paper's quintic spline)
    const double sup = (k->quintic ? 3.0 : 2.0) * p->h;
    // cells are at least sup (1 + skin) wide. A wider skin sorts less often
    // but widens the candidate search; measured per step: in 2D a skin of
    // 0.3 beats 0.1 and 0.2, with 0.4 and 0.5 within 1.5 % (41k and 1.2M
    // particles); in 3D (4.6M, FP64) 0.2 gives 8.04 ms against 8.44, 8.09,
    // 8.57 and 8.48 ms at 0.1, 0.15, 0.25 and 0.3, where the candidate ball
    // grows as its cube and the integer cell counts make the curve uneven
    const double skin = p->dim == 2 ? 0.3 : 0.2;
    const double cell_min = sup * (1.0 + skin);
    int total_bits = 0;
    double min_slack = 1e300;
    for (int d = 0; d < 3; ++d) {
        k->periodic[d] = d < p->dim ? (p->periodic[d] != 0) : 0;
        if (d >= p->dim) {
            k->nc[d] = 1;
            k->L[d] = 1.0;
            k->cs[d] = 1.0;
            k->inv_cs[d] = 1.0;
            k->halfL[d] = 0.5;
            continue;
        }
        double L = p->hi[d] - p->lo[d];
        if (!(L > 0)) return fail(SPH_EINVAL, "box axis %d has length %g", d, L);
        int nc = int(std::floor(L / cell_min));
        if (nc < 1) nc = 1;
        if (k->periodic[d] && nc < 3)
            return fail(SPH_EINVAL, "periodic axis %d needs at least 3 cells of %gh", d,
                        cell_min / p->h);
        const int max_nc = p->dim == 2 ? 65535 : 1023;
        if (nc > max_nc) return fail(SPH_EINVAL, "axis %d has %d cells (max %d)", d, nc, max_nc);
        k->nc[d] = nc;
        k->bits[d] = ceil_log2(nc);
        total_bits += k->bits[d];
        k->lo[d] = p->lo[d];
        k->L[d] = L;
        k->halfL[d] = 0.5 * L;
        k->cs[d] = L / nc;
        k->csf[d] = float(k->cs[d]);
        k->inv_cs[d] = nc / L;
        min_slack = std::fmin(min_slack, k->cs[d] - sup);
    }
    if (total_bits > 30) return fail(SPH_EINVAL, "cell grid too large (%d key bits)", total_bits);
    k->nkeys = uint32_t(1) << total_bits;
    k->sup2 = sup * sup;
    const double pi = pi_d;
    if (k->quintic)  // Sec. 2 eq:quintic-spline: 7/(478 pi h^2); in 3D the normalising 1/(120 pi h^3)
        k->wnorm = p->dim == 2 ? 7.0 / (478.0 * pi * p->h * p->h)
                               : 1.0 / (120.0 * pi * p->h * p->h * p->h);
    else
        k->wnorm = p->dim == 2 ? 7.0 / (4.0 * pi * p->h * p->h)
                               : 21.0 / (16.0 * pi * p->h * p->h * p->h);
    k->gnorm = -5.0 * k->wnorm / (p->h * p->h);
    k->inv_h = 1.0 / p->h;
    k->mass = p->dim == 2 ? p->rho0 * p->dx * p->dx : p->rho0 * p->dx * p->dx * p->dx;
    k->inv_mass = 1.0 / k->mass;
    k->rho0 = p->rho0;
    k->c = p->c;
    k->c2 = p->c * p->c;
    k->nu = p->nu;
    const double nu_edac = p->alpha * p->h * p->c / 8.0;  // Sec. 2 eq:edac-nu
    k->nu_damp = (p->flags & SPH_FLAG_DAMP_NU) ? p->nu : nu_edac;
    k->eta_h2 = p->eta * p->h * p->h;
    k->pb = p->pb;
    k->dt = p->dt;
    k->hdt = 0.5 * p->dt;
    k->disp_max = 0.999 * 0.5 * min_slack;
    {
        // candidate lists: a pair closer than sup at positions within disp_max
        // (Euclidean, the skin check of the stage updates) of the binned ones
        // is closer than sup + 2 disp_max at the binned positions (a small
        // relative margin covers rounding); capacity twice the lattice count
        // of that ball, plus slack
        const double rv = (sup + 2.0 * k->disp_max) * (1.0 + 1e-9);
        k->rv2 = rv * rv;
        const double q = rv / p->dx;
        const double ball = p->dim == 2 ? pi_d * q * q : 4.0 / 3.0 * pi_d * q * q * q;
        const double vm = 2.0 * ball + 16.0;
        k->vmax = vm < 32.0 ? 32 : (vm > 2048.0 ? 2048 : int(std::ceil(vm)));
        if (p->list_cap) k->vmax = p->list_cap;
        // measured: in 3D a list holds about a fifth of the stencil's
        // candidates and pays at every size; in 2D (about 2/5 with the 0.3
        // skin) it pays in small systems and in large FP64 ones (1.2M
        // particles: 0.998 -> 0.943 ms per step), not in large FP32 ones
        // (0.936 -> 0.942 ms)
        k->lists = (p->dim == 3 || cap < 300000 || prec == SPH_FP64) ? 1 : 0;
    }
    {
        // LDS tiles of the pair passes (on request): the first tb key bits
        // of the interleaving, 2 x 2 x 2 cells in 3D, 4 x 4 in 2D
        int tb = p->dim == 3 ? 3 : 4;
        if (tb > total_bits) tb = total_bits;
        int e[3] = {0, 0, 0};
        int maxb = 0;
        for (int a = 0; a < p->dim; ++a) maxb = k->bits[a] > maxb ? k->bits[a] : maxb;
        int pos = 0;
        for (int b = 0; b < maxb && pos < tb; ++b)
            for (int a = 0; a < p->dim && pos < tb; ++a)
                if (b < k->bits[a]) {
                    ++e[a];
                    ++pos;
                }
        k->tb = tb;
        k->nhalo = 1;
        for (int a = 0; a < 3; ++a) {
            k->text[a] = a < p->dim ? (1 << e[a]) : 1;
            k->hext[a] = a < p->dim ? k->text[a] + 2 : 1;
            k->nhalo *= k->hext[a];
        }
        k->ntiles = int64_t(k->nkeys) >> tb;
        k->tiles = (p->flags & SPH_FLAG_TILES) && k->nhalo <= kHaloCellsMax;
        k->lmax = default_maxnb(p);
    }
    k->x_inlet = p->x_inlet;
    k->x_outlet = p->x_outlet;
    k->x_outlet_end = p->x_outlet_end;
    k->inlet_len = p->inlet_len;
    k->pgate = 0.5 * p->rho0 * p->U * p->U;
    k->U = p->U;
    k->noise_amp = p->noise_amp;
    k->noise_seed = p->noise_seed;
    k->hf = float(p->h);
    k->inv_hf = float(1.0 / p->h);
    k->sup2f = float(k->sup2);
    k->wnormf = float(k->wnorm);
    k->gnormf = float(k->gnorm);
    k->massf = float(k->mass);
    k->c2f = float(k->c2);
    k->nuf = float(k->nu);
    k->nu_dampf = float(k->nu_damp);
    k->eta_h2f = float(k->eta_h2);
    k->pbf = float(k->pb);
    return SPH_OK;
}

static WsLayout layout(const Dev &k)
{
    WsLayout w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t C = size_t(k.cap);
    const size_t nscan = size_t(k.nkeys) + 2;
    w.err = take(sizeof(uint32_t));
    w.nspawn = take(sizeof(int32_t));
    w.bcount = take(sizeof(int32_t));
    w.spread = take(sizeof(uint32_t) * 3 * kSpreadStride);
    w.counts = take(sizeof(int32_t) * nscan);
    w.cell_start = take(sizeof(int32_t) * nscan);
    w.cursor = take(sizeof(int32_t) * (size_t(k.nkeys) + 1));
    w.tilesum = take(sizeof(int32_t) * size_t(tilesum_len(int64_t(nscan))));
    w.keys = take(sizeof(uint32_t) * C);
    w.scat = take(sizeof(int32_t) * C);
    w.tmp = take(sizeof(int32_t) * C);
    w.cpos = take(sizeof(uint32_t) * C);
    w.cpos_s = take(sizeof(uint32_t) * C);
    w.blist = take(sizeof(int32_t) * C);
    w.hx = take(sizeof(double) * 3 * C);  // half state (element size of FP64)
    w.hu = take(sizeof(double) * 3 * C);
    w.hut = take(sizeof(double) * 3 * C);
    w.hp = take(sizeof(double) * C);
    w.off = take(sizeof(float) * 3 * C);
    w.dragpart = take(sizeof(double) * 3 * size_t(force_grid_max(k)));
    w.sflag = take(C);
    w.stile = take(sizeof(int32_t) * size_t(nblocks(k.cap)));
    w.rebin = take(sizeof(int32_t));
    w.xbin = take(sizeof(double) * 3 * C);
    w.vfresh = take(sizeof(int32_t));
    w.vcount = take(sizeof(int32_t) * C);
    // candidate lists: rows (gather kernels) or 16-bit LDS slots (tiled search)
    w.vnbr = take(k.lists ? (k.tiles ? sizeof(uint16_t) : sizeof(int32_t)) * size_t(k.vmax) * C
                          : 0);
    // neighbour records of the force pass: FP32, or FP64 in 3D (sized for the
    // larger whatever the precision: the workspace size does not depend on it)
    w.rec = take((k.dim == 2 ? rec_bytes<2, float>() : rec_bytes<3, double>()) * C);
    // the Shepard sums (FP64, 3D FP32), from which k_pack_rec forms the
    // records and which the 2D FP64 and LDS-tiled force passes gather
    w.shep = take(sizeof(double) * C);
    // per-row flags of the reverse passes (a non-fluid neighbour)
    w.bflag = take(C);
    // LDS slots of the tiled search's table entries, read by the force pass
    w.lslot = take(k.tiles ? sizeof(uint16_t) * size_t(k.lmax) * C : 0);
    w.ttab = take(k.tiles ? sizeof(int32_t) * size_t(tile_table_ints(k)) : 0);
    // span totals of the CSR row-offset scan
    w.csum = take(sizeof(int64_t) * size_t(csr_spans(k.cap) + 1));
    w.total = off;
    return w;
}

template <typename P>
static P *at(void *ws, size_t off)
{
    return reinterpret_cast<P *>(static_cast<char *>(ws) + off);
}

static int check_state(const sph_state *s, const sph_params *p, const char *name)
{
    if (!s) return fail(SPH_EINVAL, "%s is NULL", name);
    if (s->dim != p->dim) return fail(SPH_EINVAL, "%s->dim %d != params dim %d", name, s->dim, p->dim);
    if (s->prec != SPH_FP64 && s->prec != SPH_FP32)
        return fail(SPH_EINVAL, "%s->prec must be SPH_FP64 or SPH_FP32", name);
    if (s->cap < 1 || s->cap > INT32_MAX) return fail(SPH_EINVAL, "%s->cap out of range", name);
    if (!s->n || !s->x || !s->u || !s->ut || !s->p || !s->uin || !s->ring || !s->head ||
        !s->avg || !s->jprev || !s->red_prev || !s->type || !s->id)
        return fail(SPH_EINVAL, "%s has a NULL array", name);
    return SPH_OK;
}

static int check_nlist(const sph_nlist *nl)
{
    if (!nl || !nl->count || !nl->nbr) return fail(SPH_EINVAL, "neighbour table has NULL arrays");
    if (nl->maxnb < 1 || nl->maxnb > 1024) return fail(SPH_EINVAL, "maxnb out of [1, 1024]");
    return SPH_OK;
}

static int check_derived(const sph_derived *o, bool need_drag = true)
{
    if (!o || !o->rho || !o->vol || !o->pavg || !o->a || !o->b || !o->pdot || !o->jcur ||
        !o->red || !o->force || !o->sfl || (need_drag && !o->drag))
        return fail(SPH_EINVAL, "derived output has a NULL array");
    return SPH_OK;
}

static DevState dev_state(const sph_state *s)
{
    DevState d;
    d.n = s->n;
    d.x = s->x;
    d.u = s->u;
    d.ut = s->ut;
    d.p = s->p;
    d.uin = s->uin;
    d.ring = s->ring;
    d.avg = s->avg;
    d.jprev = s->jprev;
    d.head = s->head;
    d.red_prev = s->red_prev;
    d.type = s->type;
    d.id = s->id;
    return d;
}

static DevDerived dev_derived(const sph_derived *o)
{
    DevDerived d;
    d.rho = o->rho;
    d.vol = o->vol;
    d.pavg = o->pavg;
    d.a = o->a;
    d.b = o->b;
    d.pdot = o->pdot;
    d.jcur = o->jcur;
    d.force = o->force;
    d.drag = o->drag;
    d.sfl = o->sfl;
    d.red = o->red;
    d.rec = nullptr;
    d.shep = nullptr;
    return d;
}

static DevNlist dev_nlist(const sph_nlist *nl)
{
    DevNlist d;
    d.maxnb = nl->maxnb;
    d.count = nl->count;
    d.nbr = nl->nbr;
    return d;
}

struct Ctx {
    Dev k;
    WsLayout w;
    void *ws;
    hipStream_t s;
    uint32_t *err() const { return at<uint32_t>(ws, w.err); }
    BinBufs bins() const
    {
        BinBufs b;
        b.nspawn = at<int32_t>(ws, w.nspawn);
        b.bcount = at<int32_t>(ws, w.bcount);
        b.counts = at<int32_t>(ws, w.counts);
        b.cell_start = at<int32_t>(ws, w.cell_start);
        b.cursor = at<int32_t>(ws, w.cursor);
        b.tilesum = at<int32_t>(ws, w.tilesum);
        b.scat = at<int32_t>(ws, w.scat);
        b.tmp = at<int32_t>(ws, w.tmp);
        b.blist = at<int32_t>(ws, w.blist);
        b.spread = at<uint32_t>(ws, w.spread);
        b.keys = at<uint32_t>(ws, w.keys);
        b.cpos = at<uint32_t>(ws, w.cpos);
        b.cpos_s = at<uint32_t>(ws, w.cpos_s);
        b.rebin = at<int32_t>(ws, w.rebin);
        b.xbin = at<double>(ws, w.xbin);
        b.vfresh = at<int32_t>(ws, w.vfresh);
        b.ttab = at<int32_t>(ws, w.ttab);
        return b;
    }
    Fields half() const
    {
        Fields f;
        f.x = at<double>(ws, w.hx);
        f.u = at<void>(ws, w.hu);
        f.ut = at<void>(ws, w.hut);
        f.p = at<void>(ws, w.hp);
        return f;
    }
    float *off() const { return at<float>(ws, w.off); }
    // derived buffers plus the workspace's neighbour records
    DevDerived der(const sph_derived *o) const
    {
        DevDerived d = dev_derived(o);
        // records where the force pass gathers them (Rec::USE): FP32, 3D FP64
        d.rec = k.prec == SPH_FP32 || k.dim == 3 ? at<void>(ws, w.rec) : nullptr;
        d.shep = k.prec == SPH_FP64 || k.dim == 3 ? at<void>(ws, w.shep) : nullptr;
        return d;
    }
    double *dragpart() const { return at<double>(ws, w.dragpart); }
};

static Fields fields_of(const sph_state *s)
{
    Fields f;
    f.x = s->x;
    f.u = s->u;
    f.ut = s->ut;
    f.p = s->p;
    return f;
}

static int prepare(const sph_params *p, const sph_state *st, int maxnb, void *ws,
                   size_t ws_bytes, void *stream, Ctx *c)
{
    int rc = check_state(st, p, "state");
    if (rc) return rc;
    rc = make_dev(p, st->cap, st->prec, maxnb, &c->k);
    if (rc) return rc;
    c->w = layout(c->k);
    if (force_grid(c->k) > force_grid_max(c->k))  // the drag partials are sized for the latter
        return fail(SPH_EINVAL, "internal: force grid exceeds the drag-partial buffer");
    if (!ws) return fail(SPH_EINVAL, "workspace is NULL");
    if (ws_bytes < c->w.total)
        return fail(SPH_ECAPACITY, "workspace has %zu bytes, needs %zu", ws_bytes, c->w.total);
    if (c->k.tiles && maxnb > c->k.lmax)
        return fail(SPH_EINVAL,
                    "neighbour table depth %d exceeds %d (sph_default_maxnb), which the LDS-tiled "
                    "pair passes hold per row; use a shallower table or leave SPH_FLAG_TILES off",
                    maxnb, c->k.lmax);
    c->ws = ws;
    c->s = static_cast<hipStream_t>(stream);
    return SPH_OK;
}

// Sorts *st in place: a sort gathers into *alt's buffers and the rows come
// back (one more copy); a bin that keeps the order copies nothing.
static void do_bin(Ctx &c, sph_state *st, sph_state *alt)
{
    DevState a = dev_state(st), b = dev_state(alt);
    b.n = a.n;
    launch_bin(c.k, a, b, c.bins(), c.err(), c.s);
    launch_copy_back(c.k, b, a, at<int32_t>(c.ws, c.w.vfresh), c.s);
}

// vmode: 0 stencil search; 1 first search of a step (records the candidate
// lists after a sort, else walks them); 2 walks the lists
static void do_nbrdens(Ctx &c, const sph_state *st, const Fields &R, const sph_nlist *nl,
                       const sph_derived *o, int dens, int vmode, bool clear_rebin = false,
                       float *off = nullptr)
{
    if (!c.k.lists) vmode = 0;
    VList v;
    v.fresh = at<int32_t>(c.ws, c.w.vfresh);
    v.count = at<int32_t>(c.ws, c.w.vcount);
    v.nbr = at<int32_t>(c.ws, c.w.vnbr);
    v.slot = at<uint16_t>(c.ws, c.w.vnbr);
    launch_nbrdens(c.k, dev_state(st), R, dev_nlist(nl), dens ? c.der(o) : DevDerived{},
                   dens, at<uint32_t>(c.ws, c.w.spread), at<int32_t>(c.ws, c.w.cell_start),
                   at<uint32_t>(c.ws, c.w.cpos_s), off ? off : c.off(),
                   at<uint16_t>(c.ws, c.w.lslot), at<int32_t>(c.ws, c.w.ttab),
                   clear_rebin ? at<int32_t>(c.ws, c.w.rebin) : nullptr, v, vmode, c.err(), c.s);
}

// Boundary values, then (3D) the neighbour records of the stage, which take
// the boundary rows' new values from the state (2D FP32 records are written
// by the density pass and their boundary slots by the boundary pass).
static void do_boundary(Ctx &c, const sph_state *st, const Fields &R, const sph_nlist *nl,
                        const sph_derived *o)
{
    DevDerived d = c.der(o);
    if (c.k.dim == 3) d.rec = nullptr;  // packed below
    launch_boundary(c.k, dev_state(st), R, dev_nlist(nl), d, at<int32_t>(c.ws, c.w.blist),
                    at<int32_t>(c.ws, c.w.bcount), at<uint32_t>(c.ws, c.w.spread),
                    at<int32_t>(c.ws, c.w.cell_start), c.err(), c.s);
    launch_pack_rec(c.k, dev_state(st), R, c.der(o), at<uint32_t>(c.ws, c.w.cpos_s), c.s);
}

static void do_force(Ctx &c, const sph_state *st, const Fields &R, const Fields &W,
                     const sph_nlist *nl, const sph_derived *o, int mode, double *drag,
                     double *hist, const float *off = nullptr)
{
    const int want = drag || hist;
    launch_force(c.k, dev_state(st), R, W, dev_nlist(nl), c.der(o), off ? off : c.off(),
                 at<uint32_t>(c.ws, c.w.cpos_s), at<int32_t>(c.ws, c.w.ttab),
                 at<uint16_t>(c.ws, c.w.lslot), mode, want, c.dragpart(),
                 at<double>(c.ws, c.w.xbin), at<int32_t>(c.ws, c.w.rebin), c.err(), c.s);
    if (want) launch_drag_final(c.k, c.dragpart(), drag, hist, c.s);
}

// One explicit-midpoint step (bin, two stages, end-of-step bookkeeping);
// spawned rows stay counted in the workspace until the next bin or
// launch_finish_spawn. child / events (may be NULL) record the step.
static void one_step(Ctx &c, sph_state *st, sph_state *alt, sph_nlist *nl, sph_derived *out,
                     double *hist, int32_t *child, uint8_t *events)
{
    const Fields H = c.half();
    do_bin(c, st, alt);
    const Fields M = fields_of(st);
    // stage 1 at the start state, written to the half state
    do_nbrdens(c, st, M, nl, out, 1, 1, true);
    do_boundary(c, st, M, nl, out);
    do_force(c, st, M, H, nl, out, 1, nullptr, hist);
    // stage 2 at the half state, written back over the start state
    do_nbrdens(c, st, H, nl, out, 1, 2);
    do_boundary(c, st, H, nl, out);
    do_force(c, st, H, M, nl, out, 2, nullptr, nullptr);
    launch_end_of_step(c.k, dev_state(st), dev_derived(out), at<int32_t>(c.ws, c.w.nspawn),
                       at<uint8_t>(c.ws, c.w.sflag), at<int32_t>(c.ws, c.w.stile), child, events,
                       at<int32_t>(c.ws, c.w.rebin), c.err(), c.s);
}

// Carving of the step-adjoint scratch buffer, in units of cap doubles.
struct AdjLayout {
    size_t acc_x, acc_u, acc_ut, acc_p, acc_uin, acc_ring, acc_avg, acc_jprev;
    size_t hut, jseed;
    size_t abar, bbar, pdbar, pseed, useed;
    size_t xbar, ubar, utbar, pbar, uinbar, avgbar, jprevbar;
    size_t wbar, rhobar, volbar, Pbar, Sbar, jg;
    size_t total;
};

static AdjLayout adj_layout()
{
    AdjLayout L;
    size_t o = 0;
    auto take = [&](size_t k) {
        size_t r = o;
        o += k;
        return r;
    };
    L.acc_x = take(3);
    L.acc_u = take(3);
    L.acc_ut = take(3);
    L.acc_p = take(1);
    L.acc_uin = take(3);
    L.acc_ring = take(kNavg * 4);
    L.acc_avg = take(4);
    L.acc_jprev = take(3);
    L.hut = take(3);
    L.jseed = take(3);
    L.abar = take(3);
    L.bbar = take(3);
    L.pdbar = take(1);
    L.pseed = take(1);
    L.useed = take(3);
    L.xbar = take(3);
    L.ubar = take(3);
    L.utbar = take(3);
    L.pbar = take(1);
    L.uinbar = take(3);
    L.avgbar = take(4);
    L.jprevbar = take(3);
    L.wbar = take(3);
    L.rhobar = take(1);
    L.volbar = take(1);
    L.Pbar = take(1);
    L.Sbar = take(1);
    L.jg = take(3);
    L.total = o;
    return L;
}

static DevLam dev_lam(const sph_state_adjoint *l)
{
    DevLam d;
    d.x = l->x;
    d.u = l->u;
    d.ut = l->ut;
    d.p = l->p;
    d.uin = l->uin;
    d.ring = l->ring;
    d.avg = l->avg;
    d.jprev = l->jprev;
    return d;
}

static int check_lam(const sph_state_adjoint *l, int64_t cap, const char *name)
{
    if (!l) return fail(SPH_EINVAL, "%s is NULL", name);
    if (l->cap != cap) return fail(SPH_EINVAL, "%s->cap %lld != state cap %lld", name,
                                   (long long)l->cap, (long long)cap);
    if (!l->x || !l->u || !l->ut || !l->p || !l->uin || !l->ring || !l->avg || !l->jprev)
        return fail(SPH_EINVAL, "%s has a NULL array", name);
    return SPH_OK;
}

// sph_step on a given workspace (also the static-scratch entry point's body)
int step_on_workspace(const sph_params *prm, sph_state *st, sph_state *alt, sph_nlist *nl,
                      sph_derived *out, int32_t nsteps, double *drag_hist, void *ws,
                      size_t ws_bytes, void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, nl ? nl->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl)) || (rc = check_derived(out, false))) return rc;
    rc = check_state(alt, prm, "alt");
    if (rc) return rc;
    if (alt->cap != st->cap || alt->prec != st->prec)
        return fail(SPH_EINVAL, "alt must match state in cap and precision");
    if (nsteps < 0) return fail(SPH_EINVAL, "nsteps < 0");
    launch_spread(c.k, at<uint32_t>(ws, c.w.spread), at<int32_t>(ws, c.w.rebin), c.s);
    for (int32_t s = 0; s < nsteps; ++s)
        one_step(c, st, alt, nl, out, drag_hist ? drag_hist + 3 * int64_t(s) : nullptr, nullptr,
                 nullptr);
    if (nsteps > 0) launch_finish_spawn(c.k, dev_state(st), at<int32_t>(ws, c.w.nspawn), c.s);
    return check_hip("sph_step");
}

int api_error(int code, const char *msg) { return fail(code, "%s", msg); }

}  // namespace sph

using namespace sph;

extern "C" {

const char *sph_last_error(void) { return g_err.c_str(); }

int32_t sph_default_maxnb(const sph_params *prm) { return default_maxnb(prm); }

int sph_launch_config(const sph_params *prm, int64_t cap, int32_t prec, sph_launch_info *out)
{
    if (!out) return fail(SPH_EINVAL, "out is NULL");
    Dev k;
    int rc = make_dev(prm, cap, prec, 1, &k);
    if (rc) return rc;
    for (int d = 0; d < 3; ++d) {
        out->cells[d] = k.nc[d];
        out->tile_cells[d] = k.text[d];
    }
    out->tiles = k.tiles;
    out->halo_cells = k.nhalo;
    out->group_force = force_group(k);
    out->group_search = nbr_group(k);
    out->lists = k.lists;
    return SPH_OK;
}

int sph_workspace_size(const sph_params *prm, int64_t cap, size_t *bytes)
{
    if (!bytes) return fail(SPH_EINVAL, "bytes is NULL");
    Dev k;
    int rc = make_dev(prm, cap, SPH_FP64, 1, &k);
    if (rc) return rc;
    *bytes = layout(k).total;
    return SPH_OK;
}

int sph_get_cells(const sph_params *prm, const sph_state *st, sph_cells *out, void *ws,
                  size_t ws_bytes, void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, 0, ws, ws_bytes, stream, &c);
    if (rc) return rc;
    if (!out) return fail(SPH_EINVAL, "out is NULL");
    for (int d = 0; d < 3; ++d) {
        out->ncell[d] = c.k.nc[d];
        out->cs[d] = c.k.cs[d];
    }
    out->nkeys = int64_t(c.k.nkeys);
    if (!out->cell_start && !out->key) return SPH_OK;  // sizes only: nothing to launch
    launch_cells_out(c.k, st->n, at<uint32_t>(ws, c.w.spread), at<int32_t>(ws, c.w.cell_start),
                     at<uint32_t>(ws, c.w.cpos_s), out->cell_start, out->key, c.s);
    return check_hip("sph_get_cells");
}

int64_t sph_cell_key(const sph_params *prm, int64_t cap, int32_t cx, int32_t cy, int32_t cz)
{
    Dev k;
    if (make_dev(prm, cap, SPH_FP64, 1, &k)) return -1;
    const int32_t c[3] = {cx, cy, cz};
    int maxb = 0;
    for (int a = 0; a < k.dim; ++a) {
        if (c[a] < 0 || c[a] >= k.nc[a]) return -1;
        maxb = k.bits[a] > maxb ? k.bits[a] : maxb;
    }
    if (k.dim == 2 && cz != 0) return -1;
    int64_t key = 0;
    int pos = 0;
    for (int b = 0; b < maxb; ++b)
        for (int a = 0; a < k.dim; ++a)
            if (b < k.bits[a]) {
                if ((c[a] >> b) & 1) key |= int64_t(1) << pos;
                ++pos;
            }
    return key;
}

size_t sph_workspace_bytes(const sph_params *prm, int64_t cap)
{
    size_t b = 0;
    return sph_workspace_size(prm, cap, &b) == SPH_OK ? b : 0;
}

int sph_bin(const sph_params *prm, sph_state *st, sph_state *alt, void *ws, size_t ws_bytes,
            void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, 1, ws, ws_bytes, stream, &c);
    if (rc) return rc;
    rc = check_state(alt, prm, "alt");
    if (rc) return rc;
    if (alt->cap != st->cap || alt->prec != st->prec)
        return fail(SPH_EINVAL, "alt must match state in cap and precision");
    c.k.reuse = 0;  // an explicit bin always sorts
    launch_spread(c.k, at<uint32_t>(ws, c.w.spread), at<int32_t>(ws, c.w.rebin), c.s);
    do_bin(c, st, alt);
    return check_hip("sph_bin");
}

int sph_neighbor_table(const sph_params *prm, const sph_state *st, sph_nlist *nl,
                       sph_derived *out, void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, nl ? nl->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl))) return rc;
    if (out && (rc = check_derived(out, false))) return rc;
    do_nbrdens(c, st, fields_of(st), nl, out, out != nullptr, 0);
    return check_hip("sph_neighbor_table");
}

int sph_neighbors(const sph_params *prm, const sph_state *st, sph_csr *csr, void *ws,
                  size_t ws_bytes, void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, 0, ws, ws_bytes, stream, &c);
    if (rc) return rc;
    if (!csr || !csr->row_ptr || !csr->nnz_out)
        return fail(SPH_EINVAL, "csr, csr->row_ptr and csr->nnz_out must not be NULL");
    if (csr->cap_nnz < 0) return fail(SPH_EINVAL, "csr->cap_nnz is negative");
    if (csr->cap_nnz > 0 && !csr->col) return fail(SPH_EINVAL, "csr->col is NULL");
    launch_csr(c.k, dev_state(st), at<uint32_t>(ws, c.w.spread), at<int32_t>(ws, c.w.cell_start),
               at<uint32_t>(ws, c.w.cpos_s), csr->row_ptr, csr->col, csr->cap_nnz, csr->nnz_out,
               at<int64_t>(ws, c.w.csum), c.err(), c.s);
    return check_hip("sph_neighbors");
}

int sph_density(const sph_params *prm, const sph_state *st, const sph_nlist *nl,
                sph_derived *out, void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, nl ? nl->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl)) || (rc = check_derived(out, false))) return rc;
    launch_density(c.k, dev_state(st), fields_of(st), dev_nlist(nl), c.der(out),
                   at<uint32_t>(ws, c.w.cpos_s), c.err(), c.s);
    return check_hip("sph_density");
}

int sph_outlet_extrapolate(const sph_params *prm, sph_state *st, const sph_nlist *nl,
                           sph_derived *out, void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, nl ? nl->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl)) || (rc = check_derived(out, false))) return rc;
    do_boundary(c, st, fields_of(st), nl, out);
    return check_hip("sph_outlet_extrapolate");
}

int sph_rhs(const sph_params *prm, sph_state *st, const sph_nlist *nl, sph_derived *out,
            void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, nl ? nl->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl)) || (rc = check_derived(out))) return rc;
    const Fields F = fields_of(st);
    launch_density(c.k, dev_state(st), F, dev_nlist(nl), c.der(out), at<uint32_t>(ws, c.w.cpos_s),
                   c.err(), c.s);
    do_boundary(c, st, F, nl, out);
    do_force(c, st, F, F, nl, out, 0, out->drag, nullptr);
    return check_hip("sph_rhs");
}

int sph_force(const sph_params *prm, const sph_state *st, const sph_nlist *nl,
              sph_derived *out, void *ws, size_t ws_bytes, void *stream)
{
    Ctx c;
    int rc = prepare(prm, st, nl ? nl->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl)) || (rc = check_derived(out, false))) return rc;
    const Fields F = fields_of(st);
    do_force(c, st, F, F, nl, out, 0, out->drag, nullptr);
    return check_hip("sph_force");
}

// The reverse passes differentiate the hybrid outlet with the characteristic
// inlet (either kernel).
static int hybrid_only(const sph_params *prm, const char *what)
{
    if (prm && prm->outlet != SPH_OUTLET_HYBRID)
        return fail(SPH_EUNSUPPORTED, "%s: the adjoint covers the hybrid outlet only", what);
    if (prm && (prm->flags & SPH_FLAG_MIRROR_INLET))
        return fail(SPH_EUNSUPPORTED, "%s: the adjoint covers the characteristic inlet only",
                    what);
    return SPH_OK;
}

int sph_step(const sph_params *prm, sph_state *st, sph_state *alt, sph_nlist *nl,
             sph_derived *out, int32_t nsteps, double *drag_hist, void *ws, size_t ws_bytes,
             void *stream)
{
    return step_on_workspace(prm, st, alt, nl, out, nsteps, drag_hist, ws, ws_bytes, stream);
}

int sph_step_record(const sph_params *prm, sph_state *st, sph_state *alt, sph_nlist *nl,
                    sph_derived *out, double *drag, int32_t *child, uint8_t *events, void *ws,
                    size_t ws_bytes, void *stream)
{
    if (int rc0 = hybrid_only(prm, "sph_step_record")) return rc0;
    Ctx c;
    int rc = prepare(prm, st, nl ? nl->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl)) || (rc = check_derived(out, false))) return rc;
    rc = check_state(alt, prm, "alt");
    if (rc) return rc;
    if (alt->cap != st->cap || alt->prec != st->prec)
        return fail(SPH_EINVAL, "alt must match state in cap and precision");
    if (!child || !events) return fail(SPH_EINVAL, "child and events must not be NULL");
    c.k.reuse = 0;  // the reverse pass recomputes a step from a fresh sort
    launch_spread(c.k, at<uint32_t>(ws, c.w.spread), at<int32_t>(ws, c.w.rebin), c.s);
    one_step(c, st, alt, nl, out, drag, child, events);
    launch_finish_spawn(c.k, dev_state(st), at<int32_t>(ws, c.w.nspawn), c.s);
    return check_hip("sph_step_record");
}

int sph_step_adjoint_scratch_size(const sph_params *prm, int64_t cap, size_t *bytes)
{
    if (!bytes) return fail(SPH_EINVAL, "bytes is NULL");
    Dev k;
    int rc = make_dev(prm, cap, SPH_FP64, 1, &k);
    if (rc) return rc;
    *bytes = adj_layout().total * sizeof(double) * size_t(cap);
    return SPH_OK;
}

// Checks shared by the two reverse entry points.
static int check_adjoint_args(const sph_state *st, const int32_t *child, const uint8_t *events,
                              const double fbar[3], const sph_state_adjoint *lam_next,
                              const sph_state_adjoint *lam, void *scratch,
                              size_t scratch_bytes)
{
    int rc;
    if (!child || !events || !fbar) return fail(SPH_EINVAL, "child, events, fbar must not be NULL");
    if ((rc = check_lam(lam_next, st->cap, "lam_next")) || (rc = check_lam(lam, st->cap, "lam")))
        return rc;
    const double *a[8] = {lam->x, lam->u, lam->ut, lam->p, lam->uin, lam->ring, lam->avg,
                          lam->jprev};
    const double *b[8] = {lam_next->x,   lam_next->u,    lam_next->ut,  lam_next->p,
                          lam_next->uin, lam_next->ring, lam_next->avg, lam_next->jprev};
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j)
            if (a[i] == b[j]) return fail(SPH_EINVAL, "lam and lam_next share an array");
    const size_t need = adj_layout().total * sizeof(double) * size_t(st->cap);
    if (!scratch) return fail(SPH_EINVAL, "scratch is NULL");
    if (scratch_bytes < need)
        return fail(SPH_ECAPACITY, "scratch has %zu bytes, needs %zu", scratch_bytes, need);
    return SPH_OK;
}

// Reverse of one step from its stage values: the sorted start state m / M
// (with the stage-1 boundary values), the half state H, the stage tables and
// derived values, the sort permutation and cells, and the FP32 cell offsets
// of the two stages (off1 == nullptr: rebuild those of the start state in the
// workspace before the stage-1 reverse, the workspace then holding stage 2's).
static void reverse_step(Ctx &c, const sph_state *st, const DevState &m, const Fields &M,
                         const Fields &H, const int32_t *perm, const uint32_t *cell,
                         const sph_state *work, const sph_nlist *nl1, const sph_nlist *nl2,
                         const sph_derived *d1, const sph_derived *d2, const float *off1,
                         const float *off2, const int32_t *child, const uint8_t *events,
                         const double fbar[3], const sph_state_adjoint *lam_next,
                         sph_state_adjoint *lam, void *scratch)
{
    const AdjLayout L = adj_layout();
    const size_t C = size_t(st->cap);
    double *sc = static_cast<double *>(scratch);
    auto P = [&](size_t off) { return sc + off * C; };
    StepAdj S;
    S.next = dev_lam(lam_next);
    S.out = dev_lam(lam);
    S.acc.x = P(L.acc_x);
    S.acc.u = P(L.acc_u);
    S.acc.ut = P(L.acc_ut);
    S.acc.p = P(L.acc_p);
    S.acc.uin = P(L.acc_uin);
    S.acc.ring = P(L.acc_ring);
    S.acc.avg = P(L.acc_avg);
    S.acc.jprev = P(L.acc_jprev);
    S.hut = P(L.hut);
    S.jseed = P(L.jseed);
    S.child = child;
    S.events = events;
    S.n_pre = st->n;
    DevAdj A;
    A.abar = P(L.abar);
    A.bbar = P(L.bbar);
    A.pdbar = P(L.pdbar);
    A.pseed = P(L.pseed);
    A.useed = P(L.useed);
    A.jseed = S.jseed;
    for (int d = 0; d < 3; ++d) A.fbar[d] = 0.0;
    A.xbar = P(L.xbar);
    A.ubar = P(L.ubar);
    A.utbar = P(L.utbar);
    A.pbar = P(L.pbar);
    A.uinbar = P(L.uinbar);
    A.avgbar = P(L.avgbar);
    A.jprevbar = P(L.jprevbar);
    A.wbar = P(L.wbar);
    A.rhobar = P(L.rhobar);
    A.volbar = P(L.volbar);
    A.Pbar = P(L.Pbar);
    A.Sbar = P(L.Sbar);
    A.jg = P(L.jg);
    A.bflag = at<uint8_t>(c.ws, c.w.bflag);

    launch_adj_end(c.k, m, S, A, c.s);
    launch_rhs_adjoint(c.k, m, H, dev_nlist(nl2), dev_derived(d2), A, off2, cell, c.err(), c.s);
    launch_adj_half(c.k, m, S, A, c.s);
    // the FP32 pair arithmetic reads cell-relative offsets of the stage's
    // positions: rebuild those of the start state (the same table again)
    if (!off1 && c.k.prec == SPH_FP32) do_nbrdens(c, work, M, nl1, d1, 0, 2);
    DevAdj A1 = A;
    A1.jseed = nullptr;
    for (int d = 0; d < 3; ++d) A1.fbar[d] = fbar[d];
    launch_rhs_adjoint(c.k, m, M, dev_nlist(nl1), dev_derived(d1), A1, off1 ? off1 : c.off(),
                       cell, c.err(), c.s);
    launch_adj_finish(c.k, m, dev_state(st), perm, S, A1, c.s);
}

int sph_step_adjoint(const sph_params *prm, const sph_state *st, sph_state *work,
                     const int32_t *child, const uint8_t *events, sph_nlist *nl1,
                     sph_nlist *nl2, sph_derived *d1, sph_derived *d2, const double fbar[3],
                     const sph_state_adjoint *lam_next, sph_state_adjoint *lam, void *scratch,
                     size_t scratch_bytes, void *ws, size_t ws_bytes, void *stream)
{
    if (int rc0 = hybrid_only(prm, "sph_step_adjoint")) return rc0;
    Ctx c;
    int rc = prepare(prm, st, nl1 ? nl1->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl1)) || (rc = check_nlist(nl2)) ||
        (rc = check_derived(d1, false)) || (rc = check_derived(d2, false)))
        return rc;
    if (nl1->maxnb != nl2->maxnb) return fail(SPH_EINVAL, "nl1 and nl2 differ in maxnb");
    rc = check_state(work, prm, "work");
    if (rc) return rc;
    if (work->cap != st->cap || work->prec != st->prec)
        return fail(SPH_EINVAL, "work must match state in cap and precision");
    if (work->n == st->n) return fail(SPH_EINVAL, "work needs its own live-count pointer");
    if ((rc = check_adjoint_args(st, child, events, fbar, lam_next, lam, scratch,
                                 scratch_bytes)))
        return rc;

    // recompute the step from st: bin into work (st stays untouched; the
    // live count goes to work's own pointer), then both stages
    c.k.reuse = 0;
    launch_spread(c.k, at<uint32_t>(ws, c.w.spread), at<int32_t>(ws, c.w.rebin), c.s);
    launch_adj_prep(st->n, work->n, at<int32_t>(ws, c.w.nspawn), c.s);
    DevState a = dev_state(st), b = dev_state(work);
    a.n = work->n;
    launch_bin(c.k, a, b, c.bins(), c.err(), c.s);
    const int32_t *perm = at<int32_t>(ws, c.w.tmp);  // sorted row -> row of st
    const Fields M = fields_of(work), H = c.half();
    do_nbrdens(c, work, M, nl1, d1, 1, 1);
    do_boundary(c, work, M, nl1, d1);
    do_force(c, work, M, H, nl1, d1, 1, nullptr, nullptr);
    do_nbrdens(c, work, H, nl2, d2, 1, 2);
    do_boundary(c, work, H, nl2, d2);
    do_force(c, work, H, H, nl2, d2, 0, nullptr, nullptr);

    reverse_step(c, st, dev_state(work), M, H, perm, at<uint32_t>(ws, c.w.cpos_s), work, nl1,
                 nl2, d1, d2, nullptr, c.off(), child, events, fbar, lam_next, lam, scratch);
    return check_hip("sph_step_adjoint");
}

static int check_store(const sph_step_store *sto, const sph_params *prm, const sph_state *st)
{
    if (!sto) return fail(SPH_EINVAL, "store is NULL");
    int rc = check_state(&sto->start, prm, "store->start");
    if (rc) return rc;
    if (sto->start.cap != st->cap || sto->start.prec != st->prec)
        return fail(SPH_EINVAL, "store->start must match the state in cap and precision");
    if (sto->start.n == st->n) return fail(SPH_EINVAL, "store->start needs its own live count");
    if ((rc = check_nlist(&sto->nl1)) || (rc = check_nlist(&sto->nl2)) ||
        (rc = check_derived(&sto->d1, false)) || (rc = check_derived(&sto->d2, false)))
        return rc;
    if (sto->nl1.maxnb != sto->nl2.maxnb) return fail(SPH_EINVAL, "store tables differ in maxnb");
    if (!sto->perm || !sto->cell || !sto->half_x || !sto->half_u || !sto->half_ut ||
        !sto->half_p)
        return fail(SPH_EINVAL, "store has a NULL array");
    if (st->prec == SPH_FP32 && (!sto->off1 || !sto->off2))
        return fail(SPH_EINVAL, "an FP32 store needs off1 and off2");
    return SPH_OK;
}

static Fields store_half(const sph_step_store *sto)
{
    Fields f;
    f.x = sto->half_x;
    f.u = sto->half_u;
    f.ut = sto->half_ut;
    f.p = sto->half_p;
    return f;
}

int sph_step_record_store(const sph_params *prm, sph_state *st, sph_state *alt,
                          sph_step_store *store, int32_t first, double *drag, int32_t *child,
                          uint8_t *events, void *ws, size_t ws_bytes, void *stream)
{
    if (int rc0 = hybrid_only(prm, "sph_step_record_store")) return rc0;
    Ctx c;
    int rc = prepare(prm, st, store ? store->nl1.maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_store(store, prm, st))) return rc;
    rc = check_state(alt, prm, "alt");
    if (rc) return rc;
    if (alt->cap != st->cap || alt->prec != st->prec)
        return fail(SPH_EINVAL, "alt must match state in cap and precision");
    if (!child || !events) return fail(SPH_EINVAL, "child and events must not be NULL");
    // the first step of a run sorts (spread tables and a sort request, as at
    // the start of sph_step); later ones keep the order while the skin allows
    if (first || !c.k.reuse)
        launch_spread(c.k, at<uint32_t>(ws, c.w.spread), at<int32_t>(ws, c.w.rebin), c.s);
    const bool f32 = c.k.prec == SPH_FP32;
    sph_nlist *nl1 = &store->nl1, *nl2 = &store->nl2;
    sph_derived *d1 = &store->d1, *d2 = &store->d2;
    const Fields H = store_half(store);
    // the step of one_step, with the store's tables, derived values, half
    // state and offsets, and a copy of the start state once stage 1 has set
    // its boundary values
    do_bin(c, st, alt);
    const Fields M = fields_of(st);
    do_nbrdens(c, st, M, nl1, d1, 1, 1, true, f32 ? store->off1 : nullptr);
    do_boundary(c, st, M, nl1, d1);
    do_force(c, st, M, H, nl1, d1, 1, nullptr, drag, f32 ? store->off1 : nullptr);
    launch_copy_rows(c.k, dev_state(st), dev_state(&store->start), at<int32_t>(ws, c.w.tmp),
                     at<int32_t>(ws, c.w.vfresh), store->perm, at<uint32_t>(ws, c.w.cpos_s),
                     store->cell, c.s);
    do_nbrdens(c, st, H, nl2, d2, 1, 2, false, f32 ? store->off2 : nullptr);
    do_boundary(c, st, H, nl2, d2);
    do_force(c, st, H, M, nl2, d2, 2, nullptr, nullptr, f32 ? store->off2 : nullptr);
    launch_end_of_step(c.k, dev_state(st), dev_derived(d2), at<int32_t>(c.ws, c.w.nspawn),
                       at<uint8_t>(c.ws, c.w.sflag), at<int32_t>(c.ws, c.w.stile), child, events,
                       at<int32_t>(c.ws, c.w.rebin), c.err(), c.s);
    launch_finish_spawn(c.k, dev_state(st), at<int32_t>(ws, c.w.nspawn), c.s);
    return check_hip("sph_step_record_store");
}

int sph_step_adjoint_stored(const sph_params *prm, const sph_state *st,
                            const sph_step_store *store, const int32_t *child,
                            const uint8_t *events, const double fbar[3],
                            const sph_state_adjoint *lam_next, sph_state_adjoint *lam,
                            void *scratch, size_t scratch_bytes, void *ws, size_t ws_bytes,
                            void *stream)
{
    if (int rc0 = hybrid_only(prm, "sph_step_adjoint_stored")) return rc0;
    Ctx c;
    int rc = prepare(prm, st, store ? store->nl1.maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_store(store, prm, st))) return rc;
    if ((rc = check_adjoint_args(st, child, events, fbar, lam_next, lam, scratch,
                                 scratch_bytes)))
        return rc;
    c.k.reuse = 0;
    const bool f32 = c.k.prec == SPH_FP32;
    const sph_state *work = &store->start;
    reverse_step(c, st, dev_state(work), fields_of(work), store_half(store), store->perm,
                 store->cell, work, &store->nl1, &store->nl2, &store->d1, &store->d2,
                 f32 ? store->off1 : c.off(), f32 ? store->off2 : c.off(), child, events, fbar,
                 lam_next, lam, scratch);
    return check_hip("sph_step_adjoint_stored");
}

int sph_inlet_profile_grad(const sph_params *prm, const sph_state *st,
                           const sph_state_adjoint *lam, const int32_t *index, int32_t ntheta,
                           double *grad, void *stream)
{
    int rc = check_state(st, prm, "state");
    if (rc) return rc;
    Dev k;
    if ((rc = make_dev(prm, st->cap, st->prec, 1, &k))) return rc;
    if ((rc = check_lam(lam, st->cap, "lam"))) return rc;
    if (!index || !grad) return fail(SPH_EINVAL, "index and grad must not be NULL");
    if (ntheta < 1 || ntheta > 65535) return fail(SPH_EINVAL, "ntheta must be in [1, 65535]");
    launch_profile_grad(k, st->n, dev_lam(lam), index, ntheta, grad,
                        static_cast<hipStream_t>(stream));
    return check_hip("sph_inlet_profile_grad");
}

static int rhs_adjoint_impl(const sph_params *prm, const sph_state *st, const sph_nlist *nl,
                            const sph_derived *fwd, sph_adjoint *adj, void *ws, size_t ws_bytes,
                            void *stream, bool boundary_only, const char *what);

int sph_rhs_adjoint(const sph_params *prm, const sph_state *st, const sph_nlist *nl,
                    const sph_derived *fwd, sph_adjoint *adj, void *ws, size_t ws_bytes,
                    void *stream)
{
    return rhs_adjoint_impl(prm, st, nl, fwd, adj, ws, ws_bytes, stream, false,
                            "sph_rhs_adjoint");
}

int sph_outlet_extrapolate_adjoint(const sph_params *prm, const sph_state *st,
                                   const sph_nlist *nl, const sph_derived *fwd,
                                   sph_adjoint *adj, void *ws, size_t ws_bytes, void *stream)
{
    return rhs_adjoint_impl(prm, st, nl, fwd, adj, ws, ws_bytes, stream, true,
                            "sph_outlet_extrapolate_adjoint");
}

static int rhs_adjoint_impl(const sph_params *prm, const sph_state *st, const sph_nlist *nl,
                            const sph_derived *fwd, sph_adjoint *adj, void *ws, size_t ws_bytes,
                            void *stream, bool boundary_only, const char *what)
{
    if (int rc0 = hybrid_only(prm, what)) return rc0;
    Ctx c;
    int rc = prepare(prm, st, nl ? nl->maxnb : 0, ws, ws_bytes, stream, &c);
    if (rc || (rc = check_nlist(nl)) || (rc = check_derived(fwd, false))) return rc;
    if (!adj || !adj->xbar || !adj->ubar || !adj->utbar || !adj->pbar || !adj->uinbar ||
        !adj->avgbar || !adj->scratch)
        return fail(SPH_EINVAL, "adjoint buffers have a NULL array");
    DevAdj A;
    A.abar = boundary_only ? nullptr : adj->abar;
    A.bbar = boundary_only ? nullptr : adj->bbar;
    A.pdbar = boundary_only ? nullptr : adj->pdbar;
    A.pseed = adj->pseed;
    A.useed = adj->useed;
    A.jseed = adj->jseed;
    A.jprevbar = adj->jprevbar;
    for (int d = 0; d < 3; ++d) A.fbar[d] = boundary_only ? 0.0 : adj->fbar[d];
    A.xbar = adj->xbar;
    A.ubar = adj->ubar;
    A.utbar = adj->utbar;
    A.pbar = adj->pbar;
    A.uinbar = adj->uinbar;
    A.avgbar = adj->avgbar;
    const int64_t C = st->cap;
    A.wbar = adj->scratch;             // [3][cap]
    A.rhobar = adj->scratch + 3 * C;
    A.volbar = adj->scratch + 4 * C;
    A.Pbar = adj->scratch + 5 * C;
    A.Sbar = adj->scratch + 6 * C;
    A.jg = adj->scratch + 7 * C;       // [3][cap]
    A.bflag = at<uint8_t>(c.ws, c.w.bflag);
    launch_rhs_adjoint(c.k, dev_state(st), fields_of(st), dev_nlist(nl), dev_derived(fwd), A,
                       c.off(), at<uint32_t>(c.ws, c.w.cpos_s), c.err(), c.s);
    return check_hip(what);
}

int sph_poll_error(void *ws, size_t ws_bytes, uint32_t *bits, void *stream)
{
    if (!ws || !bits) return fail(SPH_EINVAL, "NULL argument");
    if (ws_bytes < 256) return fail(SPH_EINVAL, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *err = at<uint32_t>(ws, 0);
    if (hipStreamSynchronize(s) != hipSuccess) return check_hip("sph_poll_error sync");
    uint32_t h = 0;
    if (hipMemcpy(&h, err, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
        return check_hip("sph_poll_error copy");
    const uint32_t zero = 0;
    if (hipMemcpy(err, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
        return check_hip("sph_poll_error clear");
    *bits = h;
    return check_hip("sph_poll_error");
}

int sph_live_count(const sph_state *st, int64_t *n, void *stream)
{
    if (!st || !st->n || !n) return fail(SPH_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(s) != hipSuccess) return check_hip("sph_live_count sync");
    if (hipMemcpy(n, st->n, sizeof *n, hipMemcpyDeviceToHost) != hipSuccess)
        return check_hip("sph_live_count copy");
    return SPH_OK;
}

}  // extern "C"
