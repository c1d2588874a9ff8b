/*
 * Seeded synthetic graph generators: 2D 5-point grid, 2D random geometric
 * graph (RGG) and symmetrised RMAT.  They stand in for the mesh, random
 * geometric and skewed social/web graph families of the paper's benchmark
 * sets (Section 6, "Instances"), which are not available here.
 *
 * This module only makes inputs.  It holds none of the partitioner's
 * arithmetic and is shared by the tests, the benchmark and the oracle checks.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used as a counter-based generator: the
 * i-th draw of stream `seed` is mix(seed + (i+1)*gamma).
 *
 * Output format: symmetric CSR, int32 row offsets (n+1) and int32 neighbour
 * ids, neighbours of every row strictly ascending, no self-loops, no
 * duplicates.  Weights are unit (the caller passes NULL weights).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n;
    int64_t m;          /* directed entries = xadj[n] = 2 * undirected edges */
    int32_t* xadj;
    int32_t* adjncy;
    int32_t maxdeg;
    int32_t nisolated;
} kg_graph;

static const uint64_t GAMMA = 0x9E3779B97F4A7C15ULL;

uint64_t kg_sm64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static kg_graph* alloc_graph(int32_t n, int64_t m)
{
    kg_graph* g = (kg_graph*)calloc(1, sizeof(kg_graph));
    if (!g) return NULL;
    g->n = n;
    g->m = m;
    g->xadj = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    g->adjncy = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!g->xadj || !g->adjncy) {
        free(g->xadj);
        free(g->adjncy);
        free(g);
        return NULL;
    }
    return g;
}

static void finish_stats(kg_graph* g)
{
    int32_t md = 0, iso = 0;
    for (int32_t v = 0; v < g->n; ++v) {
        int32_t d = g->xadj[v + 1] - g->xadj[v];
        if (d > md) md = d;
        if (d == 0) ++iso;
    }
    g->maxdeg = md;
    g->nisolated = iso;
}

void kg_free(kg_graph* g)
{
    if (!g) return;
    free(g->xadj);
    free(g->adjncy);
    free(g);
}

/* rows x cols 5-point grid, id = row * cols + col. */
kg_graph* kg_grid(int32_t rows, int32_t cols)
{
    if (rows < 0 || cols < 0) return NULL;
    int64_t n = (int64_t)rows * cols;
    if (n > INT32_MAX) return NULL;
    int64_t m = 2 * ((int64_t)rows * (cols > 0 ? cols - 1 : 0) + (int64_t)cols * (rows > 0 ? rows - 1 : 0));
    kg_graph* g = alloc_graph((int32_t)n, m);
    if (!g) return NULL;
    int64_t e = 0;
    g->xadj[0] = 0;
    for (int32_t r = 0; r < rows; ++r) {
        for (int32_t c = 0; c < cols; ++c) {
            int32_t id = r * cols + c;
            if (r > 0) g->adjncy[e++] = id - cols;
            if (c > 0) g->adjncy[e++] = id - 1;
            if (c + 1 < cols) g->adjncy[e++] = id + 1;
            if (r + 1 < rows) g->adjncy[e++] = id + cols;
            g->xadj[id + 1] = (int32_t)e;
        }
    }
    finish_stats(g);
    return g;
}

/* integer radius for average degree `avgdeg` in the 2^30 x 2^30 square */
int64_t kg_rgg_radius(int32_t n, double avgdeg)
{
    double r = sqrt(avgdeg / (M_PI * (double)n));
    return (int64_t)floor(r * 1073741824.0);
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/*
 * 2D random geometric graph: n points with integer coordinates in [0,2^30)^2
 * (top 30 bits of draws 2i and 2i+1), edge iff squared distance <= R^2.
 * Vertex ids are sorted by (cell_y, cell_x, point index), cell side R.
 */
kg_graph* kg_rgg(int32_t n, double avgdeg, uint64_t seed)
{
    if (n < 0) return NULL;
    int64_t R = kg_rgg_radius(n > 0 ? n : 1, avgdeg);
    if (R < 1) R = 1;
    int64_t ncell = ((1LL << 30) - 1) / R + 1;
    int64_t ncells = ncell * ncell;
    int64_t* px = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* py = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* cstart = (int64_t*)calloc((size_t)ncells + 1, sizeof(int64_t));
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t* sx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* sy = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t* deg = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
    if (!px || !py || !cell || !cstart || !order || !sx || !sy || !deg) {
        free(px); free(py); free(cell); free(cstart); free(order); free(sx); free(sy); free(deg);
        return NULL;
    }
    for (int32_t i = 0; i < n; ++i) {
        px[i] = (int64_t)(kg_sm64(seed, 2 * (uint64_t)i) >> 34);
        py[i] = (int64_t)(kg_sm64(seed, 2 * (uint64_t)i + 1) >> 34);
        cell[i] = (py[i] / R) * ncell + (px[i] / R);
        cstart[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < ncells; ++c) cstart[c + 1] += cstart[c];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncells > 0 ? ncells : 1));
        memcpy(fill, cstart, sizeof(int64_t) * (size_t)ncells);
        for (int32_t i = 0; i < n; ++i) order[fill[cell[i]]++] = i; /* stable: by point index */
        free(fill);
    }
    for (int32_t id = 0; id < n; ++id) {
        sx[id] = px[order[id]];
        sy[id] = py[order[id]];
    }
    int64_t R2 = R * R;
    /* two passes: count, then fill */
    for (int pass = 0; pass < 2; ++pass) {
        kg_graph* g = NULL;
        if (pass == 1) {
            int64_t m = 0;
            for (int32_t id = 0; id < n; ++id) m += deg[id];
            g = alloc_graph(n, m);
            if (!g) break;
            g->xadj[0] = 0;
            for (int32_t id = 0; id < n; ++id) g->xadj[id + 1] = g->xadj[id] + deg[id];
        }
        for (int32_t id = 0; id < n; ++id) {
            int64_t cx = sx[id] / R, cy = sy[id] / R;
            int32_t cnt = 0;
            int32_t* out = pass ? g->adjncy + g->xadj[id] : NULL;
            for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
                if (yy < 0 || yy >= ncell) continue;
                for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
                    if (xx < 0 || xx >= ncell) continue;
                    int64_t c = yy * ncell + xx;
                    for (int64_t p = cstart[c]; p < cstart[c + 1]; ++p) {
                        if (p == id) continue;
                        int64_t dx = sx[p] - sx[id], dy = sy[p] - sy[id];
                        if (dx * dx + dy * dy <= R2) {
                            if (pass) out[cnt] = (int32_t)p;
                            ++cnt;
                        }
                    }
                }
            }
            if (pass) qsort(out, (size_t)cnt, sizeof(int32_t), cmp_i32);
            else deg[id] = cnt;
        }
        if (pass == 1) {
            free(px); free(py); free(cell); free(cstart); free(order); free(sx); free(sy); free(deg);
            finish_stats(g);
            return g;
        }
    }
    free(px); free(py); free(cell); free(cstart); free(order); free(sx); free(sy); free(deg);
    return NULL;
}

/* LSD radix sort of 64-bit keys, `bits` significant bits, 11-bit digits. */
static int radix_sort_u64(uint64_t* a, size_t len, int bits)
{
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (len > 0 ? len : 1));
    if (!tmp) return -1;
    const int D = 11;
    size_t cnt[1 << 11];
    uint64_t* src = a;
    uint64_t* dst = tmp;
    for (int shift = 0; shift < bits; shift += D) {
        memset(cnt, 0, sizeof(cnt));
        for (size_t i = 0; i < len; ++i) cnt[(src[i] >> shift) & ((1u << D) - 1)]++;
        size_t s = 0;
        for (int d = 0; d < (1 << D); ++d) {
            size_t c = cnt[d];
            cnt[d] = s;
            s += c;
        }
        for (size_t i = 0; i < len; ++i) dst[cnt[(src[i] >> shift) & ((1u << D) - 1)]++] = src[i];
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    if (src != a) memcpy(a, src, sizeof(uint64_t) * len);
    free(tmp);
    return 0;
}

/*
 * RMAT with 2^scale vertices and `nedges` generated edges.  For edge e the
 * quadrant at recursion level i (most significant bit first) comes from the
 * top 32 bits of draw e*scale+i, compared with the integer thresholds
 * floor(a*2^32), floor((a+b)*2^32), floor((a+b+c)*2^32) where
 * (a,b,c) = (a_pct,b_pct,c_pct)/100.  No noise, no vertex permutation.  The
 * result is symmetrised; self-loops and duplicates are dropped.
 */
kg_graph* kg_rmat(int32_t scale, int64_t nedges, int32_t a_pct, int32_t b_pct, int32_t c_pct, uint64_t seed)
{
    if (scale < 1 || scale > 30 || nedges < 0) return NULL;
    int32_t n = (int32_t)1 << scale;
    uint64_t ta = ((uint64_t)a_pct << 32) / 100;
    uint64_t tb = ((uint64_t)(a_pct + b_pct) << 32) / 100;
    uint64_t tc = ((uint64_t)(a_pct + b_pct + c_pct) << 32) / 100;
    size_t cap = (size_t)nedges * 2;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (cap > 0 ? cap : 1));
    if (!keys) return NULL;
    size_t len = 0;
    for (int64_t e = 0; e < nedges; ++e) {
        uint64_t u = 0, v = 0;
        for (int32_t i = 0; i < scale; ++i) {
            uint64_t x = kg_sm64(seed, (uint64_t)e * (uint64_t)scale + (uint64_t)i) >> 32;
            uint64_t ub = 0, vb = 0;
            if (x < ta) {
            } else if (x < tb) {
                vb = 1;
            } else if (x < tc) {
                ub = 1;
            } else {
                ub = 1;
                vb = 1;
            }
            u = (u << 1) | ub;
            v = (v << 1) | vb;
        }
        if (u == v) continue;
        keys[len++] = (u << scale) | v;
        keys[len++] = (v << scale) | u;
    }
    if (radix_sort_u64(keys, len, 2 * scale) != 0) {
        free(keys);
        return NULL;
    }
    size_t w = 0;
    for (size_t i = 0; i < len; ++i)
        if (w == 0 || keys[i] != keys[w - 1]) keys[w++] = keys[i];
    kg_graph* g = alloc_graph(n, (int64_t)w);
    if (!g) {
        free(keys);
        return NULL;
    }
    uint64_t mask = ((uint64_t)1 << scale) - 1;
    memset(g->xadj, 0, sizeof(int32_t) * ((size_t)n + 1));
    for (size_t i = 0; i < w; ++i) {
        g->xadj[(keys[i] >> scale) + 1]++;
        g->adjncy[i] = (int32_t)(keys[i] & mask);
    }
    for (int32_t v = 0; v < n; ++v) g->xadj[v + 1] += g->xadj[v];
    free(keys);
    finish_stats(g);
    return g;
}
