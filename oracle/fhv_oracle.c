/*
 * CPU oracle for fragment-history volumes (Inacio and Springer,
 * arXiv 2211.15460).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, single-threaded
 * statement of what the GPU path must compute, used by the tests, the smoke
 * check and the CPU-baseline timing. No product code links or calls it, and
 * it shares no code with the GPU kernels.
 *
 * What each part follows:
 *   capture, per-pixel lists  Sec. 3.1 "Simple Layout" and Sec. 3.2 FHV_PPFL:
 *                             a pixel array holding the index of the last
 *                             inserted fragment (or -1), a global fragment
 *                             list filled through one counter, and in each
 *                             record the index of the previous fragment of
 *                             the same pixel; writes only while the counter
 *                             is below the pre-allocated size. No culling of
 *                             any kind (Sec. 3.2).
 *   capture, per-octant lists Sec. 3.1 "Octree Layout" and Sec. 3.2 FHV_POFL:
 *                             the same insertion with the head indexed by
 *                             the Morton code of the fragment's leaf octant;
 *                             each triangle is rasterized in its own tangent
 *                             frame (Sec. 3.2, Fig. 8, "1-Pass/Normal").
 *   compaction                Sec. 3.1 FHV_POFA and Sec. 3.2 FHV_POFA: per
 *                             octant a count and an offset, the offsets being
 *                             the sum of the counts of all octants before it
 *                             in Morton order; each octant's fragments stored
 *                             contiguously, with no previous index.
 *   splat                     Sec. 3.3: every fragment is projected into the
 *                             novel view, covers at least one pixel, and the
 *                             nearest fragment wins (deferred-shading
 *                             emulation).
 *   ray casting               Sec. 3.3 evaluation by ray casting: per output
 *                             pixel, every fragment the pixel's ray meets,
 *                             ordered from the viewer outward, composited
 *                             front to back with its alpha ("R/T"), or the
 *                             nearest one alone ("R"); accumulation stops at
 *                             a transmittance threshold. Written as its
 *                             definition (gather, sort, composite); the
 *                             octree traversal that finds the fragments is
 *                             the GPU's business.
 *   shading                   Sec. 5: a local illumination model per
 *                             fragment (Blinn-Phong) applied to the splat's
 *                             nearest fragments, from their packed normals.
 *   direct raster             Sec. 3.2 rasterization of the triangles
 *                             themselves in the novel view with a depth test;
 *                             the reference image for the splat.
 *
 * The paper fixes no fixed-point format, fill rule, rounding, record layout,
 * in-octant order or Morton bit order; the readings taken here are:
 *   - 16.8 fixed-point screen coordinates, samples at pixel centres,
 *     top-left fill rule for counter-clockwise triangles with y up;
 *   - every float->integer conversion rounds half to even (rint); integer
 *     interpolation (sum_k w_k a_k + floor(A/2)) / A with w_k the edge
 *     function opposite vertex k and A twice the triangle area;
 *   - 16-byte records {w0, rgba8, oct-normal, w3};
 *     PPFL w0 = depth24 | aux << 24, POFL w0 = sub-leaf x | y << 8 | z << 16
 *     | aux << 24, w3 = previous index (lists) or octant rank (arrays);
 *   - octree grid of 2^(L+8) units per cube side, tangent-plane sample
 *     spacing of 2^7 units (2^(L+1) samples per side);
 *   - Morton code with x the most significant bit of every level triple;
 *   - in-octant array order ascending by (w0, w1, w2).
 * Compile with -ffp-contract=off: every floating-point operation below is a
 * single IEEE operation in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NIL 0xFFFFFFFFu
#define DEPTH_MAX 16777215

/* ------------------------------------------------------------ helpers */

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

/* Octahedral normal packing (Cigolle et al., JCGT 2014) done with exact
 * integer arithmetic: p = n / |n|_1, folded into the upper hemisphere's
 * square when n_z < 0, each component rounded to the nearest multiple of
 * 1/32767 (halves away from zero) and stored as int16 (x low, y high).
 * A zero normal packs to 0. */
static int32_t round_snorm(int64_t num, int64_t l1) /* |num| <= l1, l1 > 0 */
{
    int64_t a = num < 0 ? -num : num;
    int64_t q = (2 * 32767 * a + l1) / (2 * l1);
    return (int32_t)(num < 0 ? -q : q);
}

uint32_t orc_oct_encode(int64_t nx, int64_t ny, int64_t nz)
{
    int64_t ax = nx < 0 ? -nx : nx, ay = ny < 0 ? -ny : ny, az = nz < 0 ? -nz : nz;
    int64_t l1 = ax + ay + az;
    int32_t qx, qy;
    if (l1 == 0) return 0;
    if (nz >= 0) {
        qx = round_snorm(nx, l1);
        qy = round_snorm(ny, l1);
    } else {
        qx = round_snorm(nx < 0 ? -(l1 - ay) : (l1 - ay), l1);
        qy = round_snorm(ny < 0 ? -(l1 - ax) : (l1 - ax), l1);
    }
    return (uint32_t)(uint16_t)(int16_t)qx | ((uint32_t)(uint16_t)(int16_t)qy << 16);
}

/* Unit normal from a packed octahedral normal, fp64. */
static void oct_decode64(uint32_t nrm, double n[3])
{
    double px = (double)(int16_t)(nrm & 0xFFFF) / 32767.0;
    double py = (double)(int16_t)(nrm >> 16) / 32767.0;
    double pz = 1.0 - fabs(px) - fabs(py);
    if (pz < 0.0) {
        double tx = (1.0 - fabs(py)) * (px >= 0.0 ? 1.0 : -1.0);
        double ty = (1.0 - fabs(px)) * (py >= 0.0 ? 1.0 : -1.0);
        px = tx;
        py = ty;
    }
    double len = sqrt(px * px + py * py + pz * pz);
    n[0] = px / len;
    n[1] = py / len;
    n[2] = pz / len;
}

void orc_oct_decode(uint32_t nrm, double* out) { oct_decode64(nrm, out); }

/* Orthonormal basis (t, b) with t x b = n from a unit normal n
 * (Duff et al., "Building an Orthonormal Basis, Revisited", JCGT 2017). */
static void onb(const double n[3], double t[3], double b[3])
{
    double s = copysign(1.0, n[2]);
    double a = -1.0 / (s + n[2]);
    double c = n[0] * n[1] * a;
    t[0] = 1.0 + s * n[0] * n[0] * a;
    t[1] = s * c;
    t[2] = -s * n[0];
    b[0] = c;
    b[1] = s + n[1] * n[1] * a;
    b[2] = -n[1];
}

void orc_tangent_frame(uint32_t nrm, double* t, double* b)
{
    double n[3];
    oct_decode64(nrm, n);
    onb(n, t, b);
}

uint64_t orc_morton3(uint32_t x, uint32_t y, uint32_t z, uint32_t levels)
{
    uint64_t k = 0;
    for (uint32_t i = 0; i < levels; ++i) {
        k |= (uint64_t)((x >> i) & 1u) << (3 * i + 2);
        k |= (uint64_t)((y >> i) & 1u) << (3 * i + 1);
        k |= (uint64_t)((z >> i) & 1u) << (3 * i);
    }
    return k;
}

static void morton3_decode(uint64_t k, uint32_t levels, uint32_t* x, uint32_t* y, uint32_t* z)
{
    *x = *y = *z = 0;
    for (uint32_t i = 0; i < levels; ++i) {
        *x |= (uint32_t)((k >> (3 * i + 2)) & 1u) << i;
        *y |= (uint32_t)((k >> (3 * i + 1)) & 1u) << i;
        *z |= (uint32_t)((k >> (3 * i)) & 1u) << i;
    }
}

/* ------------------------------------------------------- triangle raster */

/* One triangle in 16.8 fixed point with integer attributes per vertex. */
typedef struct {
    int64_t x[3], y[3];   /* 16.8 screen or tangent-plane coordinates   */
    int64_t attr[3][7];   /* up to 7 integer attributes per vertex       */
    int n_attr;
} tri_fx;

typedef void (*emit_fn)(void* user, int64_t sx, int64_t sy, const int64_t* attr);

/* Twice the signed area of (v0, v1, v2). */
static int64_t area2(const tri_fx* t)
{
    return (t->x[1] - t->x[0]) * (t->y[2] - t->y[0]) - (t->y[1] - t->y[0]) * (t->x[2] - t->x[0]);
}

/* Edge function of the directed edge i->j at point (px, py): positive on
 * the left of the edge. */
static int64_t edge(const tri_fx* t, int i, int j, int64_t px, int64_t py)
{
    return (t->x[j] - t->x[i]) * (py - t->y[i]) - (t->y[j] - t->y[i]) * (px - t->x[i]);
}

/* Top-left rule for a counter-clockwise triangle with y up: a sample on the
 * edge i->j belongs to the triangle when the edge runs downwards (a left
 * edge) or runs horizontally towards -x (a top edge). */
static int owns_edge(const tri_fx* t, int i, int j)
{
    int64_t dy = t->y[j] - t->y[i], dx = t->x[j] - t->x[i];
    return dy < 0 || (dy == 0 && dx < 0);
}

/* Rasterize one triangle over the sample lattice (256 i + 128, 256 j + 128),
 * i in [i_lo, i_hi], j in [j_lo, j_hi]; samples are visited row by row
 * (j ascending, then i ascending) and every covered one is emitted with its
 * interpolated attributes. Both windings are rasterized (no culling);
 * attributes stay with their vertices. */
static void raster_tri(const tri_fx* tin, int64_t i_lo, int64_t i_hi, int64_t j_lo, int64_t j_hi,
                       emit_fn emit, void* user)
{
    tri_fx t = *tin;
    int64_t A = area2(&t);
    if (A == 0) return;
    if (A < 0) { /* swap v1 and v2, attributes travel with the vertices */
        int64_t s;
        s = t.x[1]; t.x[1] = t.x[2]; t.x[2] = s;
        s = t.y[1]; t.y[1] = t.y[2]; t.y[2] = s;
        for (int a = 0; a < t.n_attr; ++a) { s = t.attr[1][a]; t.attr[1][a] = t.attr[2][a]; t.attr[2][a] = s; }
        A = -A;
    }
    int64_t xmin = t.x[0], xmax = t.x[0], ymin = t.y[0], ymax = t.y[0];
    for (int k = 1; k < 3; ++k) {
        if (t.x[k] < xmin) xmin = t.x[k];
        if (t.x[k] > xmax) xmax = t.x[k];
        if (t.y[k] < ymin) ymin = t.y[k];
        if (t.y[k] > ymax) ymax = t.y[k];
    }
    int64_t bi0 = floor_div(xmin - 128, 256), bi1 = floor_div(xmax - 128, 256) + 1;
    int64_t bj0 = floor_div(ymin - 128, 256), bj1 = floor_div(ymax - 128, 256) + 1;
    if (bi0 < i_lo) bi0 = i_lo;
    if (bi1 > i_hi) bi1 = i_hi;
    if (bj0 < j_lo) bj0 = j_lo;
    if (bj1 > j_hi) bj1 = j_hi;
    int own01 = owns_edge(&t, 0, 1), own12 = owns_edge(&t, 1, 2), own20 = owns_edge(&t, 2, 0);
    int64_t half = A / 2;
    for (int64_t j = bj0; j <= bj1; ++j) {
        for (int64_t i = bi0; i <= bi1; ++i) {
            int64_t px = 256 * i + 128, py = 256 * j + 128;
            int64_t e01 = edge(&t, 0, 1, px, py);
            int64_t e12 = edge(&t, 1, 2, px, py);
            int64_t e20 = edge(&t, 2, 0, px, py);
            if (!(e01 > 0 || (e01 == 0 && own01))) continue;
            if (!(e12 > 0 || (e12 == 0 && own12))) continue;
            if (!(e20 > 0 || (e20 == 0 && own20))) continue;
            /* weight of vertex k = edge function of the edge opposite k */
            int64_t out[7];
            for (int a = 0; a < t.n_attr; ++a) {
                __int128 num = (__int128)e12 * t.attr[0][a] + (__int128)e20 * t.attr[1][a] +
                               (__int128)e01 * t.attr[2][a];
                out[a] = (int64_t)((num + half) / A);
            }
            emit(user, i, j, out);
        }
    }
}

static void rgba_split(uint32_t c, int64_t* out)
{
    for (int k = 0; k < 4; ++k) out[k] = (c >> (8 * k)) & 0xFF;
}

static uint32_t rgba_join(const int64_t* c)
{
    return (uint32_t)c[0] | ((uint32_t)c[1] << 8) | ((uint32_t)c[2] << 16) | ((uint32_t)c[3] << 24);
}

/* ------------------------------------------------------- list insertion */

typedef struct {
    uint32_t* head;
    uint32_t* pool;  /* uint32[4 * cap] */
    uint64_t cap;
    uint64_t counter;
    uint64_t key_lo, key_hi; /* POFL: only keys in [key_lo, key_hi) are kept */
    /* current triangle */
    uint32_t aux, nrm;
    uint32_t width;  /* PPFL */
    uint32_t levels; /* POFL */
    int mode;
} lists_t;

/* Append one fragment to the list of `key` (Sec. 3.2): take the next index
 * from the counter; only when it is below the capacity store the record with
 * the previous head as its link and make it the new head. */
static void insert(lists_t* L, uint64_t key, uint32_t w0, uint32_t w1, uint32_t w2)
{
    uint64_t idx = L->counter++;
    if (idx >= L->cap) return;
    uint32_t* r = L->pool + 4 * idx;
    r[0] = w0;
    r[1] = w1;
    r[2] = w2;
    r[3] = L->head[key];
    L->head[key] = (uint32_t)idx;
}

static void emit_ppfl(void* user, int64_t i, int64_t j, const int64_t* a)
{
    lists_t* L = (lists_t*)user;
    uint64_t key = (uint64_t)j * L->width + (uint64_t)i;
    uint32_t w0 = (uint32_t)a[0] | (L->aux << 24);
    insert(L, key, w0, rgba_join(a + 1), L->nrm);
}

/* Per-pixel capture (FHV_PPFL), orthographic view along -z of clip space.
 * Vertices are clip-space xyz in [-1,1]; the pixel (px, py) has its sample at
 * the pixel centre, y up. head must hold W*H entries set to -1 by the caller
 * (NIL); pool holds 4*cap words. Returns the number of fragments produced,
 * which exceeds cap on overflow. */
uint64_t orc_capture_ppfl(const float* pos, const uint32_t* rgba, const uint32_t* tri,
                          const uint8_t* obj, uint32_t n_tri, uint32_t width, uint32_t height,
                          uint32_t* head, uint32_t* pool, uint64_t cap)
{
    lists_t L = {head, pool, cap, 0, 0, UINT64_MAX, 0, 0, width, 0, 0};
    for (uint32_t t = 0; t < n_tri; ++t) {
        tri_fx f;
        int64_t q[3][3];
        int skip = 0;
        f.n_attr = 5;
        for (int k = 0; k < 3; ++k) {
            const float* p = pos + 3 * (size_t)tri[3 * t + k];
            double x = p[0], y = p[1], z = p[2];
            if (!(fabs(x) <= 64.0 && fabs(y) <= 64.0 && fabs(z) <= 64.0)) skip = 1;
            f.x[k] = (int64_t)rint((x + 1.0) * (width * 128.0));
            f.y[k] = (int64_t)rint((y + 1.0) * (height * 128.0));
            double zd = rint((z + 1.0) * 0.5 * (double)DEPTH_MAX);
            if (zd < 0.0) zd = 0.0;
            if (zd > (double)DEPTH_MAX) zd = (double)DEPTH_MAX;
            f.attr[k][0] = (int64_t)zd;
            rgba_split(rgba[tri[3 * t + k]], &f.attr[k][1]);
            /* normal from vertices snapped to a 2^-20 lattice */
            q[k][0] = (int64_t)rint(x * 1048576.0);
            q[k][1] = (int64_t)rint(y * 1048576.0);
            q[k][2] = (int64_t)rint(z * 1048576.0);
        }
        int64_t ux = q[1][0] - q[0][0], uy = q[1][1] - q[0][1], uz = q[1][2] - q[0][2];
        int64_t vx = q[2][0] - q[0][0], vy = q[2][1] - q[0][1], vz = q[2][2] - q[0][2];
        if (skip) continue;
        L.nrm = orc_oct_encode(uy * vz - uz * vy, uz * vx - ux * vz, ux * vy - uy * vx);
        L.aux = obj ? obj[t] : 0;
        raster_tri(&f, 0, (int64_t)width - 1, 0, (int64_t)height - 1, emit_ppfl, &L);
    }
    return L.counter;
}

static void emit_pofl(void* user, int64_t i, int64_t j, const int64_t* a)
{
    (void)i;
    (void)j;
    lists_t* L = (lists_t*)user;
    uint32_t px = (uint32_t)a[0], py = (uint32_t)a[1], pz = (uint32_t)a[2];
    uint64_t key = orc_morton3(px >> 8, py >> 8, pz >> 8, L->levels);
    if (key < L->key_lo || key >= L->key_hi) return;
    uint32_t w0 = (px & 0xFF) | ((py & 0xFF) << 8) | ((pz & 0xFF) << 16) | (L->aux << 24);
    insert(L, key - L->key_lo, w0, rgba_join(a + 3), L->nrm);
}

/* Per-octant capture (FHV_POFL) with tangent-space rasterization. Vertices
 * lie in the scene cube [0,1)^3 and snap to the grid of G = 2^(L+8) units per
 * side. Each triangle is rasterized in the plane of its packed normal with
 * the frame of Duff et al.; the sample lattice has a spacing of 2^7 grid
 * units and is anchored at the projection of the grid origin. Each sample's
 * grid position is interpolated from the vertices; its leaf is the top L bits
 * per axis. head holds 8^L entries set to NIL by the caller. */
uint64_t orc_capture_pofl_proj(const float* pos, const uint32_t* rgba, const uint32_t* tri,
                               const uint8_t* obj, uint32_t n_tri, uint32_t levels, uint32_t proj,
                               uint64_t key_lo, uint64_t key_hi, uint32_t* head, uint32_t* pool,
                               uint64_t cap);

uint64_t orc_capture_pofl(const float* pos, const uint32_t* rgba, const uint32_t* tri,
                          const uint8_t* obj, uint32_t n_tri, uint32_t levels,
                          uint32_t* head, uint32_t* pool, uint64_t cap)
{
    return orc_capture_pofl_proj(pos, rgba, tri, obj, n_tri, levels, 0, 0, (uint64_t)1 << (3 * levels),
                                 head, pool, cap);
}

/* Per-octant capture keeping only the fragments whose key lies in
 * [key_lo, key_hi): the lists of exactly those keys, with head[key - key_lo]
 * (the octree of a large scene taken one key range at a time). The counter
 * counts the kept fragments only. */
uint64_t orc_capture_pofl_range(const float* pos, const uint32_t* rgba, const uint32_t* tri,
                                const uint8_t* obj, uint32_t n_tri, uint32_t levels, uint64_t key_lo,
                                uint64_t key_hi, uint32_t* head, uint32_t* pool, uint64_t cap)
{
    return orc_capture_pofl_proj(pos, rgba, tri, obj, n_tri, levels, 0, key_lo, key_hi, head, pool, cap);
}

/* The capture with a choice of rasterization plane (Sec. 3.2, Figs. 7-8,
 * Table 2): proj 0 the triangle's own plane ("1-Pass/Normal", above);
 * 1 the x-y plane, seen along z ("1-Pass/View"); 2 and 3 the y-z, z-x and
 * x-y planes, every triangle rasterized once in each ("3-Pass/1-Way" and
 * "1-Pass/3-Way" capture the same fragments; only their order differs, and
 * the order is not part of the result). In an axis plane the sample
 * coordinates are two of the grid coordinates, in cyclic order after the
 * axis, scaled to the lattice of 2^7 grid units; a triangle seen edge-on
 * there has zero area and no fragments. */
uint64_t orc_capture_pofl_proj(const float* pos, const uint32_t* rgba, const uint32_t* tri,
                               const uint8_t* obj, uint32_t n_tri, uint32_t levels, uint32_t proj,
                               uint64_t key_lo, uint64_t key_hi, uint32_t* head, uint32_t* pool,
                               uint64_t cap)
{
    lists_t L = {head, pool, cap, 0, key_lo, key_hi, 0, 0, 0, levels, 1};
    const int64_t G = (int64_t)1 << (levels + 8);
    const double Gd = (double)G;
    for (uint32_t t = 0; t < n_tri; ++t) {
        int64_t P[3][3];
        int skip = 0;
        for (int k = 0; k < 3; ++k) {
            const float* p = pos + 3 * (size_t)tri[3 * t + k];
            for (int c = 0; c < 3; ++c) {
                if (!isfinite(p[c])) skip = 1;
                double g = isfinite(p[c]) ? floor((double)p[c] * Gd) : 0.0;
                if (g < 0.0) g = 0.0;
                if (g > Gd - 1.0) g = Gd - 1.0;
                P[k][c] = (int64_t)g;
            }
        }
        if (skip) continue;
        int64_t ux = P[1][0] - P[0][0], uy = P[1][1] - P[0][1], uz = P[1][2] - P[0][2];
        int64_t vx = P[2][0] - P[0][0], vy = P[2][1] - P[0][1], vz = P[2][2] - P[0][2];
        int64_t nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
        if (nx == 0 && ny == 0 && nz == 0) continue; /* degenerate: no fragments */
        uint32_t nrm = orc_oct_encode(nx, ny, nz);
        L.nrm = nrm;
        L.aux = obj ? obj[t] : 0;
        tri_fx f;
        f.n_attr = 7;
        for (int k = 0; k < 3; ++k) {
            f.attr[k][0] = P[k][0];
            f.attr[k][1] = P[k][1];
            f.attr[k][2] = P[k][2];
            rgba_split(rgba[tri[3 * t + k]], &f.attr[k][3]);
        }
        if (proj == 0) {
            double n[3], tt[3], bb[3];
            oct_decode64(nrm, n);
            onb(n, tt, bb);
            for (int k = 0; k < 3; ++k) {
                double px = (double)P[k][0], py = (double)P[k][1], pz = (double)P[k][2];
                double u = px * tt[0] + py * tt[1] + pz * tt[2];
                double v = px * bb[0] + py * bb[1] + pz * bb[2];
                /* 2^7 grid units per sample = 256 sub-sample units: scale by 2 */
                f.x[k] = (int64_t)rint(2.0 * u);
                f.y[k] = (int64_t)rint(2.0 * v);
            }
            raster_tri(&f, INT64_MIN / 4, INT64_MAX / 4, INT64_MIN / 4, INT64_MAX / 4, emit_pofl, &L);
            continue;
        }
        /* axis planes: seen along z only (View), or along x, y and z */
        for (int axis = 0; axis < 3; ++axis) {
            if (proj == 1 && axis != 2) continue;
            int cu = (axis + 1) % 3, cv = (axis + 2) % 3;
            for (int k = 0; k < 3; ++k) {
                f.x[k] = 2 * P[k][cu];
                f.y[k] = 2 * P[k][cv];
            }
            raster_tri(&f, INT64_MIN / 4, INT64_MAX / 4, INT64_MIN / 4, INT64_MAX / 4, emit_pofl, &L);
        }
    }
    return L.counter;
}

/* ------------------------------------------------------------ compaction */

static int cmp_rec(const void* a, const void* b)
{
    const uint32_t* x = (const uint32_t*)a;
    const uint32_t* y = (const uint32_t*)b;
    for (int k = 0; k < 3; ++k) {
        if (x[k] < y[k]) return -1;
        if (x[k] > y[k]) return 1;
    }
    return 0;
}

/* Per-octant arrays from per-octant (or per-pixel) lists. For every key in
 * ascending order: its count is the length of its list, its offset is the
 * sum of the counts of all smaller keys, and its records are stored at
 * [offset, offset + count) ascending by (w0, w1, w2), with w3 set to the
 * octant's rank among occupied keys. The occupied table gets (key, offset,
 * count) per occupied key; table entries at rank >= cap_occ are not stored.
 * Only pool indices below min(counter, cap) are valid list members.
 * Returns the number of occupied keys; frag must hold 4*min(counter, cap)
 * words. Returns UINT64_MAX if a list is malformed (cycle or bad index). */
uint64_t orc_compact(const uint32_t* head, uint64_t n_head, const uint32_t* pool, uint64_t counter,
                     uint64_t cap, uint64_t* oct_key, uint32_t* oct_off, uint32_t* oct_cnt,
                     uint64_t cap_occ, uint32_t* frag)
{
    uint64_t F = counter < cap ? counter : cap;
    uint64_t off = 0, rank = 0;
    for (uint64_t key = 0; key < n_head; ++key) {
        uint64_t cnt = 0;
        for (uint32_t i = head[key]; i != NIL; i = pool[4 * (uint64_t)i + 3]) {
            if ((uint64_t)i >= F || off + cnt >= F) return UINT64_MAX;
            memcpy(frag + 4 * (off + cnt), pool + 4 * (uint64_t)i, 16);
            ++cnt;
        }
        if (cnt == 0) continue;
        qsort(frag + 4 * off, cnt, 16, cmp_rec);
        for (uint64_t k = 0; k < cnt; ++k) frag[4 * (off + k) + 3] = (uint32_t)rank;
        if (rank < cap_occ) {
            oct_key[rank] = key;
            oct_off[rank] = (uint32_t)off;
            oct_cnt[rank] = (uint32_t)cnt;
        }
        off += cnt;
        ++rank;
    }
    return rank;
}

/* ------------------------------------------------------------ splat */

static uint32_t f32_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static float bits_f32(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* Position of array fragment `i` in the view's input space.
 * PPFL (mode 0): (px + 1/2, py + 1/2, depth24) with the pixel from the key.
 * POFL (mode 1): grid units, leaf from the key, sub-leaf offset from w0,
 * plus 1/2. */
static void frag_pos(int mode, uint32_t width, uint32_t levels, uint64_t key, uint32_t w0, float* p)
{
    if (mode == 0) {
        uint32_t px = (uint32_t)(key % width), py = (uint32_t)(key / width);
        p[0] = (float)px + 0.5f;
        p[1] = (float)py + 0.5f;
        p[2] = (float)(w0 & 0xFFFFFF);
    } else {
        uint32_t x, y, z;
        morton3_decode(key, levels, &x, &y, &z);
        p[0] = (float)((x << 8) | (w0 & 0xFF)) + 0.5f;
        p[1] = (float)((y << 8) | ((w0 >> 8) & 0xFF)) + 0.5f;
        p[2] = (float)((z << 8) | ((w0 >> 16) & 0xFF)) + 0.5f;
    }
}

/* Point splat of the per-octant arrays into n_views views (Sec. 3.3).
 * m: n_views row-major fp32 3x4 matrices; each row is evaluated as
 * ((m0*x + m1*y) + m2*z) + m3 in fp32. Fragment i covers the k x k pixel
 * square whose lower-left pixel is floor(s + 1/2 - k/2) per axis; per pixel
 * the fragment with the smallest (depth bits, index) wins; fragments with
 * depth <= 0 or NaN are skipped. Uncovered pixels keep colour 0, depth 0,
 * coverage 0. zbuf: u64 [V][H][W] scratch; outputs [V][H][W]. */
void orc_splat(int mode, uint32_t width_cap, uint32_t levels, const uint64_t* oct_key, uint64_t n_keys,
               const uint32_t* frag, uint64_t n_frag, const float* m, const uint32_t* wh_k,
               uint32_t n_views, uint64_t* zbuf, uint32_t* out_rgba, float* out_depth,
               uint8_t* out_cov)
{
    size_t base = 0;
    for (uint32_t v = 0; v < n_views; ++v) {
        uint32_t W = wh_k[3 * v], H = wh_k[3 * v + 1], k = wh_k[3 * v + 2];
        const float* M = m + 12 * v;
        uint64_t* z = zbuf + base;
        for (size_t p = 0; p < (size_t)W * H; ++p) z[p] = ~(uint64_t)0;
        float c = 0.5f - 0.5f * (float)k;
        for (uint64_t i = 0; i < n_frag; ++i) {
            const uint32_t* r = frag + 4 * i;
            float p[3], s[3];
            if (r[3] >= n_keys) continue; /* octant row not stored: not drawn */
            frag_pos(mode, width_cap, levels, oct_key[r[3]], r[0], p);
            for (int row = 0; row < 3; ++row) {
                float a = M[4 * row + 0] * p[0];
                float b = M[4 * row + 1] * p[1];
                float e = M[4 * row + 2] * p[2];
                s[row] = ((a + b) + e) + M[4 * row + 3];
            }
            if (!(s[2] > 0.0f)) continue;
            float fx = floorf(s[0] + c), fy = floorf(s[1] + c);
            if (!(fx > -1073741824.0f && fx < 1073741824.0f)) continue;
            if (!(fy > -1073741824.0f && fy < 1073741824.0f)) continue;
            int64_t x0 = (int64_t)fx, y0 = (int64_t)fy;
            uint64_t key = ((uint64_t)f32_bits(s[2]) << 32) | (uint32_t)i;
            for (int64_t y = y0; y < y0 + (int64_t)k; ++y) {
                if (y < 0 || y >= (int64_t)H) continue;
                for (int64_t x = x0; x < x0 + (int64_t)k; ++x) {
                    if (x < 0 || x >= (int64_t)W) continue;
                    uint64_t* d = z + (size_t)y * W + (size_t)x;
                    if (key < *d) *d = key;
                }
            }
        }
        for (size_t p = 0; p < (size_t)W * H; ++p) {
            if (z[p] == ~(uint64_t)0) {
                out_rgba[base + p] = 0;
                out_depth[base + p] = 0.0f;
                out_cov[base + p] = 0;
            } else {
                uint32_t id = (uint32_t)(z[p] & 0xFFFFFFFFu);
                out_rgba[base + p] = frag[4 * (size_t)id + 1];
                out_depth[base + p] = bits_f32((uint32_t)(z[p] >> 32));
                out_cov[base + p] = 1;
            }
        }
        base += (size_t)W * H;
    }
}

/* ------------------------------------------------------------ ray casting */

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Ray casting of the per-octant arrays into one view (Sec. 3.3, evaluation
 * by ray casting). The view is orthographic (the matrix m as in orc_splat):
 * the ray of pixel (x, y) meets fragment i when i projects into that pixel,
 * floor(s) = (x, y) per axis, with depth s2 > 0 (the one-pixel footprint of
 * the splat). The fragments a pixel's ray meets are ordered by (depth bits,
 * index) and composited front to back in fp32, each operation in the order
 * written:
 *   a = A / 255 (mode 1; mode 0 takes a = 1), w = T * a,
 *   C_c = C_c + w * (c / 255) for c = R, G, B, T = T * (1 - a),
 * starting from C = 0, T = 1 and stopping after the fragment that leaves
 * T < tau or T = 0 (later fragments add exact zeros). Output per pixel: (C_r, C_g, C_b, 1 - T), zero where no fragment
 * is met. out: float [H][W][4]. Returns the largest number of fragments
 * met by one pixel. */
uint64_t orc_raycast(uint32_t levels, const uint64_t* oct_key, const uint32_t* frag, uint64_t n_frag,
                     const float* m, uint32_t W, uint32_t H, int mode, float tau, float* out)
{
    size_t np = (size_t)W * H;
    uint64_t* cnt = (uint64_t*)calloc(np + 1, sizeof(uint64_t));
    int64_t* pix = (int64_t*)malloc((n_frag ? n_frag : 1) * sizeof(int64_t));
    uint64_t* key = (uint64_t*)malloc((n_frag ? n_frag : 1) * sizeof(uint64_t));
    /* every fragment's pixel (or none) and sort key */
    for (uint64_t i = 0; i < n_frag; ++i) {
        const uint32_t* r = frag + 4 * i;
        float p[3], s[3];
        pix[i] = -1;
        frag_pos(1, 0, levels, oct_key[r[3]], r[0], p);
        for (int row = 0; row < 3; ++row) {
            float a = m[4 * row + 0] * p[0];
            float b = m[4 * row + 1] * p[1];
            float e = m[4 * row + 2] * p[2];
            s[row] = ((a + b) + e) + m[4 * row + 3];
        }
        if (!(s[2] > 0.0f)) continue;
        float fx = floorf(s[0]), fy = floorf(s[1]);
        if (!(fx >= 0.0f && fx < (float)W && fy >= 0.0f && fy < (float)H)) continue;
        pix[i] = (int64_t)fy * W + (int64_t)fx;
        key[i] = ((uint64_t)f32_bits(s[2]) << 32) | (uint32_t)i;
        cnt[pix[i] + 1] += 1;
    }
    /* group by pixel (counting sort), then order each group */
    for (size_t q = 0; q < np; ++q) cnt[q + 1] += cnt[q];
    uint64_t* list = (uint64_t*)malloc((cnt[np] ? cnt[np] : 1) * sizeof(uint64_t));
    uint64_t* fill = (uint64_t*)malloc((np ? np : 1) * sizeof(uint64_t));
    memcpy(fill, cnt, np * sizeof(uint64_t));
    for (uint64_t i = 0; i < n_frag; ++i)
        if (pix[i] >= 0) list[fill[pix[i]]++] = key[i];
    uint64_t deepest = 0;
    for (size_t q = 0; q < np; ++q) {
        uint64_t b = cnt[q], n = cnt[q + 1] - b;
        float* o = out + 4 * q;
        o[0] = o[1] = o[2] = o[3] = 0.0f;
        if (n == 0) continue;
        if (n > deepest) deepest = n;
        qsort(list + b, n, sizeof(uint64_t), cmp_u64);
        float c[3] = {0.0f, 0.0f, 0.0f}, t = 1.0f;
        for (uint64_t j = 0; j < n; ++j) {
            uint32_t id = (uint32_t)(list[b + j] & 0xFFFFFFFFu);
            uint32_t rgba = frag[4 * (size_t)id + 1];
            float a = mode == 1 ? (float)(rgba >> 24) / 255.0f : 1.0f;
            float w = t * a;
            for (int k = 0; k < 3; ++k) c[k] = c[k] + w * ((float)((rgba >> (8 * k)) & 0xFFu) / 255.0f);
            t = t * (1.0f - a);
            if (t < tau || t == 0.0f) break;
        }
        o[0] = c[0];
        o[1] = c[1];
        o[2] = c[2];
        o[3] = 1.0f - t;
    }
    free(cnt);
    free(pix);
    free(key);
    free(list);
    free(fill);
    return deepest;
}

/* ------------------------------------------------------------ shading */

/* Blinn-Phong shading of the splat's winners (Sec. 5: a local illumination
 * model per fragment, Phong 1975 / Blinn 1977), fp32, each operation in the
 * order written:
 *   normal: p = (int16 x, int16 y) / 32767, z = (1 - |px|) - |py|; when
 *   z < 0 the octahedron's lower half unfolds, (px, py) = ((1 - |py|) s(px),
 *   (1 - |px|) s(py)) with s(0) = +1; n = (px, py, z) / sqrt((px^2 + py^2) +
 *   z^2);
 *   two-sided: if n.V < 0 the normal is flipped (n.X = (nx Xx + ny Xy) + nz Xz);
 *   d = max(n.L, 0), s = (n.L > 0 ? max(n.H, 0) : 0) squared `shine`
 *   times (exponent 2^shine), c = albedo (R, G, B / 255):
 *   out = c * (ka + kd * d) + ks * s, alpha 1; empty pixels stay 0.
 * light: per view L[3], V[3], H[3] (unit light, viewer and half vectors,
 * given), ka, kd, ks, and shine as a float. zbuf: the splat's
 * [V][H][W] keys (depth bits << 32 | index, ~0 empty). out: [V][H][W][4]. */
void orc_shade(const uint32_t* frag, const uint64_t* zbuf, uint64_t n_pix_per_view, uint32_t n_views,
               const float* light, float* out)
{
    for (uint32_t v = 0; v < n_views; ++v) {
        const float* P = light + 13 * v;
        const float *Lv = P, *Vv = P + 3, *Hv = P + 6;
        const float ka = P[9], kd = P[10], ks = P[11];
        const int shine = (int)P[12];
        for (uint64_t q = 0; q < n_pix_per_view; ++q) {
            const uint64_t z = zbuf[v * n_pix_per_view + q];
            float* o = out + 4 * (v * n_pix_per_view + q);
            o[0] = o[1] = o[2] = o[3] = 0.0f;
            if (z == ~(uint64_t)0) continue;
            const uint32_t* r = frag + 4 * (size_t)(uint32_t)z;
            const uint32_t w2 = r[2], c = r[1];
            float px = (float)(int16_t)(w2 & 0xFFFF) / 32767.0f;
            float py = (float)(int16_t)(w2 >> 16) / 32767.0f;
            const float nz = (1.0f - fabsf(px)) - fabsf(py);
            if (nz < 0.0f) {
                const float tx = (1.0f - fabsf(py)) * (px >= 0.0f ? 1.0f : -1.0f);
                const float ty = (1.0f - fabsf(px)) * (py >= 0.0f ? 1.0f : -1.0f);
                px = tx;
                py = ty;
            }
            const float len = sqrtf((px * px + py * py) + nz * nz);
            float n[3] = {px / len, py / len, nz / len};
            const float ndv = (n[0] * Vv[0] + n[1] * Vv[1]) + n[2] * Vv[2];
            if (ndv < 0.0f) {
                n[0] = -n[0];
                n[1] = -n[1];
                n[2] = -n[2];
            }
            const float ndl = (n[0] * Lv[0] + n[1] * Lv[1]) + n[2] * Lv[2];
            const float ndh = (n[0] * Hv[0] + n[1] * Hv[1]) + n[2] * Hv[2];
            const float d = ndl > 0.0f ? ndl : 0.0f;
            float sp = (ndl > 0.0f && ndh > 0.0f) ? ndh : 0.0f;
            for (int k = 0; k < shine; ++k) sp = sp * sp;
            for (int k = 0; k < 3; ++k) {
                const float al = (float)((c >> (8 * k)) & 0xFFu) / 255.0f;
                o[k] = al * (ka + kd * d) + ks * sp;
            }
            o[3] = 1.0f;
        }
    }
}

/* ------------------------------------------------------------ direct raster */

typedef struct {
    uint64_t* zbuf;  /* (depth24 << 32) | triangle, smaller wins */
    uint32_t* col;
    uint32_t W, H;
    uint32_t t;
} draster_t;

static void emit_direct(void* user, int64_t i, int64_t j, const int64_t* a)
{
    draster_t* D = (draster_t*)user;
    size_t p = (size_t)j * D->W + (size_t)i;
    uint64_t key = ((uint64_t)a[0] << 32) | D->t;
    if (key < D->zbuf[p]) {
        D->zbuf[p] = key;
        D->col[p] = rgba_join(a + 1);
    }
}

/* Direct rasterization of the triangles into one view with a depth test:
 * the reference image a novel-view reconstruction is judged against.
 * mode 0: vertices in clip space, mapped to the capture window units
 * (px + 1/2 at pixel centres, depth24) before the view matrix; mode 1:
 * vertices in [0,1)^3, scaled to grid units (2^(L+8) per side). The view
 * matrix m (fp32 3x4) is applied in fp64; screen x, y are snapped to 16.8
 * fixed point and the depth row (in [1,2)) is quantized to depth24 as
 * rint((d - 1) * (2^24 - 1)). Per pixel the smallest (depth24, triangle) wins.
 * Outputs: rgba (0 where uncovered), depth (fp32 of the winning depth24
 * mapped back to [1,2], 0 where uncovered), coverage 0/1. */
void orc_direct_raster(int mode, uint32_t cap_w, uint32_t cap_h, uint32_t levels,
                       const float* pos, const uint32_t* rgba, const uint32_t* tri,
                       uint32_t n_tri, const float* m, uint32_t W, uint32_t H,
                       uint64_t* zbuf, uint32_t* out_rgba, float* out_depth, uint8_t* out_cov)
{
    draster_t D = {zbuf, out_rgba, W, H, 0};
    for (size_t p = 0; p < (size_t)W * H; ++p) {
        zbuf[p] = ~(uint64_t)0;
        out_rgba[p] = 0;
    }
    double G = (double)((int64_t)1 << (levels + 8));
    for (uint32_t t = 0; t < n_tri; ++t) {
        tri_fx f;
        f.n_attr = 5;
        int bad = 0;
        for (int k = 0; k < 3; ++k) {
            const float* p = pos + 3 * (size_t)tri[3 * t + k];
            double w[3];
            if (mode == 0) {
                w[0] = (p[0] + 1.0) * (cap_w * 0.5);
                w[1] = (p[1] + 1.0) * (cap_h * 0.5);
                w[2] = (p[2] + 1.0) * 0.5 * (double)DEPTH_MAX;
            } else {
                w[0] = p[0] * G;
                w[1] = p[1] * G;
                w[2] = p[2] * G;
            }
            double s[3];
            for (int r = 0; r < 3; ++r)
                s[r] = (double)m[4 * r] * w[0] + (double)m[4 * r + 1] * w[1] +
                       (double)m[4 * r + 2] * w[2] + (double)m[4 * r + 3];
            if (!(fabs(s[0]) < 1048576.0 && fabs(s[1]) < 1048576.0)) bad = 1;
            f.x[k] = (int64_t)rint(s[0] * 256.0);
            f.y[k] = (int64_t)rint(s[1] * 256.0);
            double zd = rint((s[2] - 1.0) * (double)DEPTH_MAX);
            if (zd < 0.0) zd = 0.0;
            if (zd > (double)DEPTH_MAX) zd = (double)DEPTH_MAX;
            f.attr[k][0] = (int64_t)zd;
            rgba_split(rgba[tri[3 * t + k]], &f.attr[k][1]);
        }
        if (bad) continue;
        D.t = t;
        raster_tri(&f, 0, (int64_t)W - 1, 0, (int64_t)H - 1, emit_direct, &D);
    }
    for (size_t p = 0; p < (size_t)W * H; ++p) {
        if (zbuf[p] == ~(uint64_t)0) {
            out_depth[p] = 0.0f;
            out_cov[p] = 0;
        } else {
            out_depth[p] = (float)(1.0 + (double)(zbuf[p] >> 32) / (double)DEPTH_MAX);
            out_cov[p] = 1;
        }
    }
}

/* ------------------------------------------------------------ PSNR */

/* PSNR over the R, G, B bytes of two RGBA8 images, MAX = 255, the mean
 * squared error taken over 3 * n_pix values. Identical images give +inf. */
double orc_psnr_rgb(const uint32_t* a, const uint32_t* b, uint64_t n_pix)
{
    double se = 0.0;
    for (uint64_t p = 0; p < n_pix; ++p)
        for (int c = 0; c < 3; ++c) {
            double d = (double)((a[p] >> (8 * c)) & 0xFF) - (double)((b[p] >> (8 * c)) & 0xFF);
            se += d * d;
        }
    double mse = se / (3.0 * (double)n_pix);
    if (mse == 0.0) return INFINITY;
    return 10.0 * log10(255.0 * 255.0 / mse);
}
