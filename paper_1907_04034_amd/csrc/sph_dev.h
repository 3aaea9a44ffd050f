// sph_dev.h -- device-side helpers shared by the gfx950 kernels of libsph.
//
// Everything here is wave64 / CDNA4 code. Per-particle arrays are
// component-major ([comp][cap]) so that one wave reads 64 consecutive
// elements of a component in one coalesced transaction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sph.h"

namespace sph {

constexpr int kBlock = 256;        // 4 waves of 64
constexpr int kNavg = 6;           // time-average window (Sec. 3.4, eq:N)
constexpr int64_t kIdGeneration = int64_t(1) << 40;

// Constants derived once per call on the host and passed by value.
struct Dev {
    int dim, flags, maxnb, prec;
    int reuse;           // keep the last bin while the skin allows (sph_step only)
    int outlet;          // SPH_OUTLET_* rule
    int quintic;         // 1: the paper's quintic spline (support 3h), 0: Wendland C2 (2h)
    int g_force, g_nbr;  // lanes per target requested (0 = automatic)
    int periodic[3];
    int nc[3];          // cells per axis
    int bits[3];        // Morton bits per axis
    uint32_t nkeys;     // 2^(sum bits); key nkeys marks a dead particle
    int64_t cap;
    double lo[3], L[3], halfL[3], cs[3], inv_cs[3];
    float csf[3];
    double h, inv_h, sup2, wnorm, gnorm, mass, inv_mass, rho0, c, c2, nu, nu_damp, eta_h2, pb;
    double dt, hdt, disp_max;
    double rv2;  // squared radius of the step path's candidate lists
    int vmax;    // candidate-list entries per particle
    int lists;   // the step path keeps candidate lists (else it searches the stencil)
    // LDS tiles of the pair passes: a tile is an aligned block of 2^tb Morton
    // keys, a box of text[a] cells per axis; its halo (the tile grown by one
    // cell on every side) holds every neighbour of the tile's rows
    int tiles;          // 1: the neighbour search and force pass use the tiled kernels
    int tb;             // key bits per tile
    int text[3];        // tile extent per axis (cells)
    int hext[3];        // halo extent per axis (text + 2)
    int nhalo;          // halo cells per tile (product of hext)
    int64_t ntiles;     // nkeys >> tb
    int lmax;           // depth of the tiled search's LDS-slot table (the default table depth)
    double x_inlet, x_outlet, x_outlet_end, inlet_len, pgate, U, noise_amp;
    uint64_t noise_seed;
    float hf, inv_hf, sup2f, wnormf, gnormf, massf, c2f, nuf, nu_dampf, eta_h2f, pbf;
};

// LDS capacity of the tiled kernels, in halo rows (rows past it are read
// from global memory): the search stages FP64 positions, the force pass the
// FP32 neighbour record or the FP64 fields x, u, ut, p, rho, V and the kind.
constexpr int kHaloCellsMax = 128;
__host__ __device__ constexpr int tile_cap_search(int dim) { return dim == 3 ? 1024 : 512; }
__host__ __device__ constexpr int tile_cap_force(int dim, int prec)
{
    return prec == SPH_FP32 ? (dim == 3 ? 1024 : 512) : (dim == 3 ? 768 : 384);
}

// Device pointers of one state (element type of the real fields depends on
// the precision).
struct DevState {
    int64_t *n;
    double *x;
    void *u, *ut, *p;
    double *uin, *ring, *avg, *jprev;
    uint8_t *head, *red_prev, *type;
    int64_t *id;
};

// The four fields a right-hand side reads at its stage (x, u, ut, p) and the
// fields a stage update writes; the start-of-step state and the half state
// each provide one.
struct Fields {
    double *x;
    void *u, *ut, *p;
};

struct DevDerived {
    void *rho, *vol, *pavg, *a, *b, *pdot;
    double *jcur, *force, *drag, *sfl;
    uint8_t *red;
    void *rec;  // neighbour records of the force pass (Rec, rec_chunk)
    // the Shepard sums S of the density pass (FP64 and 3D FP32), from which
    // the 3D records are packed and the 2D FP64 and LDS-tiled force passes
    // form a neighbour's rho = m S and V = 1/S
    void *shep;
};

// Neighbour record: what the force pass gathers of a neighbour j, packed so
// that it arrives in a few 16-byte loads instead of one load per field
// (positions or FP32 cell offsets, p, u, w = ut - u, rho and V or the Shepard
// sum S, kind and, in FP32, the packed cell), in the state's element type;
// slots in T units. 3D records are written after the boundary pass by
// k_pack_rec, 2D FP32 ones by the density pass with the boundary pass
// updating the slots of the values it sets; 2D FP64 has none (Rec::USE). FP64
// records (96 bytes) hold S, from which a neighbour's rho = m S and V = 1/S
// are formed per pair by the operations that give the stored fields, so the
// values are the same. In 3D FP32 the record is
// packed into 48 bytes: the Shepard sum S stands for rho = m S (formed per
// pair as the density pass forms the stored field) and V = 1/S (per pair by
// the hardware reciprocal, within about an ulp of the stored field, like the
// other FP32 pair divisions) and the kind's class (kind_class) shares the word of
// the 30-bit packed cell: three 16-byte loads instead of four (measured on
// the 4.6M-particle duct: force pass 1.26 -> 1.19 ms).
template <int DIM, typename T>
struct Rec {
    static constexpr bool F32 = sizeof(T) == 4;
    static constexpr bool PACKED = F32 && DIM == 3;
    // the Shepard sum S in place of rho and V (FP64 and 3D FP32)
    static constexpr bool SREC = PACKED || !F32;
    // chunk-major (FP64) or row-major (FP32) storage, see rec_chunk
    static constexpr bool CM = !F32;  // (3D FP32 measured the same either way)
    // the force pass gathers records (FP32, 3D FP64) or, in 2D FP64, the
    // state's fields and the Shepard sum (measured: 2D FP64 records left the
    // 1.2M-particle cylinder's force pass at 168 us and the pass that writes
    // them cost more than they saved, 0.850 -> 0.873 ms per step)
    static constexpr bool USE = F32 || DIM == 3;
    static constexpr int X = 0, P = DIM, U = 4, RHO = SREC ? -1 : 3, W = DIM == 3 ? 7 : 6,
                         VOL = DIM == 3 ? 10 : (F32 ? 8 : 3),  // SREC: S
                         AUX = DIM == 3 ? 11 : (F32 ? 9 : 8);
    // FP32: cell bits and kind bits (one word when PACKED); FP64: kind
    static constexpr int USED = F32 && !PACKED ? AUX + 2 : AUX + 1;
    static constexpr int PER = 16 / int(sizeof(T));    // T per 16-byte chunk
    static constexpr int NC = (USED + PER - 1) / PER;  // chunks that carry data
    static constexpr int N = NC * PER;                 // row stride in T (row-major)
};


// What the force pass distinguishes of a neighbour's kind: fluid, inlet or
// outlet (and rows already marked dead), slip wall, no-slip wall or body.
__device__ inline uint32_t kind_class(int t)
{
    return t == SPH_FLUID ? 0u : t == SPH_WALL_SLIP ? 2u
                             : (t == SPH_WALL_NOSLIP || t == SPH_BODY) ? 3u : 1u;
}
__device__ inline int class_kind(uint32_t c)
{
    return c == 0u ? SPH_FLUID : c == 2u ? SPH_WALL_SLIP : c == 3u ? SPH_WALL_NOSLIP : SPH_INLET;
}
constexpr uint32_t kCellBits = 0x3FFFFFFFu;  // the 3D packed cell (3 x 10 bits)
template <int DIM, typename T>
inline size_t rec_bytes() { return sizeof(T) * Rec<DIM, T>::N; }

template <typename T>
struct Chunk;
template <>
struct Chunk<float> {
    using V = float4;
    __device__ static inline void get(const V &c, float *v) { v[0] = c.x; v[1] = c.y; v[2] = c.z; v[3] = c.w; }
    __device__ static inline V make(const float *v) { return V{v[0], v[1], v[2], v[3]}; }
};
template <>
struct Chunk<double> {
    using V = double2;
    __device__ static inline void get(const V &c, double *v) { v[0] = c.x; v[1] = c.y; }
    __device__ static inline V make(const double *v) { return V{v[0], v[1]}; }
};

// Chunk ch (16 bytes) of row j's record. FP32 records are row-major (a row's
// chunks together); FP64 records are chunk-major (chunk ch of every row
// together, at ch * cap + j), so that the chunks of neighbouring rows share
// cache lines: a wave's gather of neighbour chunks then touches about 30
// 64-byte lines per instruction against 46 for a row-major record and 23 per
// field for the state's own arrays, 6 chunk loads against 13 field loads per
// neighbour in 3D. (FP32 records measured the same either way: that pass is
// bound by its arithmetic.)
template <int DIM, typename T>
__device__ inline typename Chunk<T>::V *rec_chunk(void *rec, int64_t cap, int64_t j, int ch)
{
    using L = Rec<DIM, T>;
    auto *b = reinterpret_cast<typename Chunk<T>::V *>(rec);
    return L::CM ? b + (int64_t(ch) * cap + j) : b + (j * L::NC + ch);
}
template <int DIM, typename T>
__device__ inline T *rec_slot(void *rec, int64_t cap, int64_t j, int slot)
{
    using L = Rec<DIM, T>;
    return reinterpret_cast<T *>(rec_chunk<DIM, T>(rec, cap, j, slot / L::PER)) + slot % L::PER;
}

// kind and packed cell stored in record slots (bit copies in FP32)
template <typename T>
__device__ inline T rec_word(uint32_t w);
template <>
__device__ inline float rec_word<float>(uint32_t w) { return __uint_as_float(w); }
template <>
__device__ inline double rec_word<double>(uint32_t w) { return double(w); }
template <typename T>
__device__ inline uint32_t rec_uint(T v);
template <>
__device__ inline uint32_t rec_uint<float>(float v) { return __float_as_uint(v); }
template <>
__device__ inline uint32_t rec_uint<double>(double v) { return uint32_t(v); }

// Objective weights and gradient buffers of the reverse pass: the weights on
// a, b, pdot in the state's element type, every other array FP64; pair
// arithmetic in the state's precision.
struct DevAdj {
    const void *abar, *bbar, *pdbar;
    const double *pseed, *useed;  // adjoints seeded on boundary values (non-fluid rows)
    const double *jseed;          // adjoint seeded on the characteristic values J
    double fbar[3];
    double *xbar, *ubar, *utbar, *pbar, *uinbar, *avgbar, *jprevbar;
    double *wbar, *rhobar, *volbar, *Pbar, *Sbar, *jg;
    // per row: 1 if a neighbour is not fluid (or unknown), written by the pair
    // reverse; a fluid row with 0 has no boundary neighbour to gather from in
    // the boundary reverse (null: every row walks its neighbours)
    uint8_t *bflag = nullptr;
};

// Logical block for hardware block blockIdx.x when nb_logical blocks are
// needed: the 8 XCDs (which receive consecutive hardware blocks round-robin)
// each get one contiguous range of logical blocks. Returns -1 for hardware
// blocks beyond the need.
__device__ inline int64_t xcd_block(int64_t nb_logical)
{
    const int64_t per = (nb_logical + 7) / 8;
    const int64_t b = blockIdx.x;
    if (b / 8 >= per) return -1;
    const int64_t lb = (b % 8) * per + b / 8;
    return lb < nb_logical ? lb : -1;
}

inline int xcd_grid(int64_t nb_logical) { return int(((nb_logical + 7) / 8) * 8); }

template <int G, typename V>
__device__ inline V gsum(V v)
{
#pragma unroll
    for (int m = G / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, G);
    return v;
}

// Exclusive prefix sum of one value per thread over a block of kBlock
// threads (lds: kBlock entries); *total receives the block sum.
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *lds, int32_t *total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const int32_t add = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const int32_t incl = lds[t];
    *total = lds[kBlock - 1];
    __syncthreads();
    return incl - v;
}

// events of one row at the end of a step, recorded for the reverse pass
constexpr uint8_t kEvPush = SPH_EV_PUSH, kEvToOutlet = SPH_EV_TO_OUTLET,
                  kEvDelete = SPH_EV_DELETE, kEvSpawn = SPH_EV_SPAWN;

// adjoint of a particle state, laid out like the state ([comp][cap])
struct DevLam {
    double *x, *u, *ut, *p, *uin, *ring, *avg, *jprev;
};

// buffers of the reverse of one step
struct StepAdj {
    DevLam next;  // adjoint of the state after the step (its row order)
    DevLam acc;   // accumulators of the sorted start state
    DevLam out;   // adjoint of the state before the step (its row order)
    double *hut;                 // direct adjoint of the half-state ut
    double *jseed;               // adjoint of the stage-2 characteristic values
    const int32_t *child;
    const uint8_t *events;
    const int64_t *n_pre;  // rows of the state before the step
};

struct DevNlist {
    int32_t maxnb;
    int32_t *count, *nbr;
};

// Candidate lists of the step path: for every particle the members of its
// 3^d stencil within Dev::rv2 of it at the last sort (binned positions), in
// stencil order. While every particle stays within disp_max per axis of its
// binned position (checked by the stage updates), each pair closer than 2h is
// in these lists, so a search may walk them instead of the stencil.
struct VList {
    const int32_t *fresh;  // 1: the step's bin sorted (rebuild the lists)
    int32_t *count;        // entries per particle; -1: overflowed, search the stencil
    int32_t *nbr;          // [cap][vmax] rows (gather kernels)
    uint16_t *slot;        // [cap][vmax] LDS slots of the tile halos (tiled search)
};

// Workspace carving (byte offsets from the workspace base).
struct WsLayout {
    size_t err, nspawn, bcount, spread, counts, cell_start, cursor, tilesum, keys, scat, tmp,
        cpos, cpos_s, blist, hx, hu, hut, hp, off, dragpart, sflag, stile, rebin, xbin, vfresh, vcount,
        vnbr, rec, shep, bflag, lslot, ttab, csum, total;
};

__host__ __device__ inline bool is_wall(int t)
{
    return t == SPH_WALL_SLIP || t == SPH_WALL_NOSLIP || t == SPH_BODY;
}

// ------------------------------------------------------------------ kernel
// Wendland C2 quintic with support 2h: W = a (1 - q/2)^4 (2q + 1),
// grad_i W_ij = F (r_i - r_j) with F = -5 a (1 - q/2)^3 / h^2.
template <typename T>
__device__ inline T wendland_w(T q, T wnorm)
{
    T t = T(1) - T(0.5) * q;
    T t2 = t * t;
    return q < T(2) ? wnorm * t2 * t2 * (T(2) * q + T(1)) : T(0);
}

template <typename T>
__device__ inline T wendland_f(T q, T gnorm)  // gnorm = -5 a / h^2
{
    T t = T(1) - T(0.5) * q;
    return q < T(2) ? gnorm * t * t * t : T(0);
}

// The paper's quintic spline (Sec. 2 eq:quintic-spline), support 3h:
// W = a [(3-q)^5 - 6 (2-q)^5 + 15 (1-q)^5], each power taken as zero past its
// range; F = W'(r)/r = (-5 a / h^2) [(3-q)^4 - 6 (2-q)^4 + 15 (1-q)^4] / q,
// where for q < 1 the bracket over q is the polynomial 24 - 24 q^2 + 10 q^3
// (no division near q = 0). a = 7/(478 pi h^2) in 2D, 1/(120 pi h^3) in 3D.
template <typename T>
__device__ inline T pow5(T t)
{
    const T t2 = t * t;
    return t2 * t2 * t;
}

template <typename T>
__device__ inline T quintic_w(T q, T wnorm)
{
    const T t3 = q < T(3) ? T(3) - q : T(0);
    const T t2 = q < T(2) ? T(2) - q : T(0);
    const T t1 = q < T(1) ? T(1) - q : T(0);
    return wnorm * (pow5(t3) - T(6) * pow5(t2) + T(15) * pow5(t1));
}

template <typename T>
__device__ inline T quintic_f(T q, T gnorm)  // gnorm = -5 a / h^2
{
    if (q < T(1)) {
        const T q2 = q * q;
        return gnorm * (T(24) - T(24) * q2 + T(10) * q2 * q);
    }
    const T t3 = q < T(3) ? T(3) - q : T(0);
    const T t2 = q < T(2) ? T(2) - q : T(0);
    const T a3 = t3 * t3, a2 = t2 * t2;
    return gnorm * (a3 * a3 - T(6) * a2 * a2) / q;
}

// (dF/dr)/r, needed by the reverse passes: Wendland C2 -1.5 gnorm t^2 / (h^2 q)
// with t = 1 - q/2; quintic spline gnorm (-48 + 30 q) / h^2 for q < 1 and
// gnorm (P' q - P) / (h^2 q^3) with P = (3-q)^4 - 6 (2-q)^4 beyond (each
// power zero past its range), the derivative of F over r.
template <typename T>
__device__ inline T wendland_g(T q, T gnorm, T inv_h)
{
    const T t = T(1) - T(0.5) * q;
    return q < T(2) ? T(-1.5) * gnorm * t * t * inv_h * inv_h / q : T(0);
}

template <typename T>
__device__ inline T quintic_g(T q, T gnorm, T inv_h)
{
    if (q < T(1)) return gnorm * (T(-48) + T(30) * q) * inv_h * inv_h;
    const T t3 = q < T(3) ? T(3) - q : T(0);
    const T t2 = q < T(2) ? T(2) - q : T(0);
    const T P = t3 * t3 * t3 * t3 - T(6) * t2 * t2 * t2 * t2;
    const T dP = T(-4) * (t3 * t3 * t3 - T(6) * t2 * t2 * t2);
    return gnorm * (dP * q - P) * inv_h * inv_h / (q * q * q);
}

// The run's kernel (the flag is uniform over a launch).
template <typename T>
__device__ inline T kernel_g(const Dev &k, T q, T gnorm, T inv_h)
{
    return k.quintic ? quintic_g<T>(q, gnorm, inv_h) : wendland_g<T>(q, gnorm, inv_h);
}

template <typename T>
__device__ inline T kernel_w(const Dev &k, T q, T wnorm)
{
    return k.quintic ? quintic_w<T>(q, wnorm) : wendland_w<T>(q, wnorm);
}

template <typename T>
__device__ inline T kernel_f(const Dev &k, T q, T gnorm)
{
    return k.quintic ? quintic_f<T>(q, gnorm) : wendland_f<T>(q, gnorm);
}

// ------------------------------------------------------------------ geometry
// Minimum-image difference and its square, FP64, summed left to right with
// contraction disabled: the neighbour predicate must be bitwise reproducible.
__device__ inline double min_image(double v, int per, double L, double half)
{
    if (per) {
        if (v > half) v -= L;
        else if (v < -half) v += L;
    }
    return v;
}

template <int DIM>
__device__ inline double dist2_exact(const Dev &k, const double *xi, const double *xj,
                                     double r[3])
{
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        r[d] = min_image(xi[d] - xj[d], k.periodic[d], k.L[d], k.halfL[d]);
    }
    s = r[0] * r[0];
    s = s + r[1] * r[1];
    if (DIM == 3) s = s + r[2] * r[2];
    return s;
}

// Packed integer cell coordinates: 2D 16 bits per axis, 3D 10 bits per axis.
template <int DIM>
__host__ __device__ inline uint32_t pack_cell(const int c[3])
{
    if (DIM == 2) return uint32_t(c[0]) | (uint32_t(c[1]) << 16);
    return uint32_t(c[0]) | (uint32_t(c[1]) << 10) | (uint32_t(c[2]) << 20);
}

template <int DIM>
__host__ __device__ inline void unpack_cell(uint32_t p, int c[3])
{
    if (DIM == 2) {
        c[0] = int(p & 0xFFFFu);
        c[1] = int(p >> 16);
        c[2] = 0;
    } else {
        c[0] = int(p & 0x3FFu);
        c[1] = int((p >> 10) & 0x3FFu);
        c[2] = int(p >> 20);
    }
}

// Morton key from per-axis "spread" tables: spread[d * kSpreadStride + c] is
// the coordinate c with its bits moved to the key positions of axis d.
constexpr int kSpreadStride = 1 << 16;  // entries per axis table (2D axes up to 65536)

template <int DIM>
__device__ inline uint32_t morton_key(const uint32_t *spread, const int c[3])
{
    uint32_t k = spread[c[0]] | spread[kSpreadStride + c[1]];
    if (DIM == 3) k |= spread[2 * kSpreadStride + c[2]];
    return k;
}

__device__ inline void raise_error(uint32_t *err, uint32_t bit) { atomicOr(err, bit); }

template <typename T>
__device__ inline T ld(const void *p, int64_t i)
{
    return static_cast<const T *>(p)[i];
}
template <typename T>
__device__ inline void st(void *p, int64_t i, T v)
{
    static_cast<T *>(p)[i] = v;
}

__device__ inline bool bad_index(int32_t j, int64_t n) { return uint64_t(j) >= uint64_t(n); }

// FP32 offset of position x from the corner of cell c along axis d (c is the
// row's cell at the last sort). On a periodic axis the position is taken at
// its image nearest that cell: a row that crossed the face since the sort was
// wrapped into the box by its stage update while its cell stayed on the far
// side, and the plain difference would be off by the box length.
__device__ inline float cell_offset(const Dev &k, int d, double x, int c)
{
    double o = x - (k.lo[d] + double(c) * k.cs[d]);
    if (k.periodic[d]) {
        if (o > k.halfL[d]) o -= k.L[d];
        else if (o < -k.halfL[d]) o += k.L[d];
    }
    return float(o);
}

// Pair separation r_i - r_j in the arithmetic type. FP64: minimum image of
// the absolute positions. FP32: cell-relative offsets plus the (wrapped)
// cell difference times the cell size, so no large coordinate is rounded to
// FP32.
template <int DIM, typename T>
struct Sep;

template <int DIM>
struct Sep<DIM, double> {
    double xi[3];
    __device__ inline void load_i(const Dev &k, const Fields &R, const float *, const uint32_t *,
                                  int64_t i)
    {
        xi[2] = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) xi[d] = R.x[d * k.cap + i];
    }
    __device__ inline double get(const Dev &k, const Fields &R, const float *, const uint32_t *,
                                 int64_t j, double r[3]) const
    {
        double xj[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) xj[d] = R.x[d * k.cap + j];
        return dist2_exact<DIM>(k, xi, xj, r);
    }
    // the same from a neighbour record's slots (positions at Rec::X)
    __device__ inline double get_rec(const Dev &k, const double *v, double r[3]) const
    {
        double xj[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) xj[d] = v[d];
        return dist2_exact<DIM>(k, xi, xj, r);
    }
};

template <int DIM>
struct Sep<DIM, float> {
    float oi[3];
    int ci[3];
    __device__ inline void load_i(const Dev &k, const Fields &, const float *off,
                                  const uint32_t *cpos, int64_t i)
    {
        oi[2] = 0.f;
        unpack_cell<DIM>(cpos[i], ci);
#pragma unroll
        for (int d = 0; d < DIM; ++d) oi[d] = off[d * k.cap + i];
    }
    __device__ inline float get(const Dev &k, const Fields &, const float *off,
                                const uint32_t *cpos, int64_t j, float r[3]) const
    {
        int cj[3];
        unpack_cell<DIM>(cpos[j], cj);
        float s = 0.f;
        r[2] = 0.f;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            int dc = ci[d] - cj[d];
            if (k.periodic[d]) {
                if (dc > 1) dc -= k.nc[d];
                else if (dc < -1) dc += k.nc[d];
            }
            r[d] = (oi[d] - off[d * k.cap + j]) + float(dc) * k.csf[d];
            s += r[d] * r[d];
        }
        return s;
    }
    // the same from a neighbour record: offsets at Rec::X, packed cell cpj
    __device__ inline float get_rec(const Dev &k, const float *v, uint32_t cpj, float r[3]) const
    {
        int cj[3];
        unpack_cell<DIM>(cpj, cj);
        float s = 0.f;
        r[2] = 0.f;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            int dc = ci[d] - cj[d];
            if (k.periodic[d]) {
                if (dc > 1) dc -= k.nc[d];
                else if (dc < -1) dc += k.nc[d];
            }
            r[d] = (oi[d] - v[d]) + float(dc) * k.csf[d];
            s += r[d] * r[d];
        }
        return s;
    }
};

}  // namespace sph
