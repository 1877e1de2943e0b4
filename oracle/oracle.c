/*
 * FP64 CPU oracle for the TreePM gravity hot path of the Arepo code
 * (Weinberger, Springel & Pakmor, "The AREPO public code release", ApJS 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no source,
 * header, table or helper with the HIP library and includes none of it.
 *
 * It is written to be read against the paper, not to be fast:
 *   - root cube, integer coordinates, Peano-Hilbert keys   (Sec. 3.1, Sec. 8)
 *   - octree by sequential insertion of single particles   (Sec. 3.1)
 *   - monopole moments computed recursively                 (Sec. 3.1)
 *   - per-target recursive walk with the relative and the
 *     geometric opening criteria and the 1.2 L box rule     (Sec. 3.1)
 *   - spline softening, zero-lag potential -Gm/eps,
 *     Newtonian beyond 2.8 eps                              (Sec. 3.2)
 *   - short-range truncation and cutoff of the tree force   (Sec. 3.4)
 *   - particle-mesh long-range force: CIC, FFT Poisson
 *     solve with Gaussian filter and deconvolution,
 *     finite differences, interpolation                     (Sec. 3.3, 3.4)
 *   - the same for isolated systems: zero-padded mesh and the
 *     real-space long-range Green's function                (Sec. 3.3)
 * plus the exact references the method is checked against: direct O(N^2)
 * summation and an Ewald sum for periodic boxes (Sec. 3.1, Ewald paragraph).
 *
 * Readings of points the paper leaves open:
 *   - curve: Skilling's transpose-form Hilbert algorithm (2004), 21 bits per
 *     axis, key interleaved from the most significant bit, x-major;
 *   - maximum depth 21 (63-bit keys); particles with equal 21-bit integer
 *     coordinates share one depth-21 cell, ordered by particle index (the
 *     paper's randomly chosen neighbour sub-node is not reproducible);
 *   - children are visited in Peano-Hilbert order;
 *   - the 1.2 L box rule is applied under both criteria;
 *   - a node is discarded under TreePM when the distance from the target to
 *     the node's cube exceeds the cutoff; a particle counts when r < r_cut;
 *   - the printed short-range factor of Sec. 3.4 has the sign of its
 *     exponent and its role garbled: the short-range force factor is
 *     erfc(r/2rs) + r/(sqrt(pi) rs) exp(-r^2/4rs^2) and the long-range
 *     factor is one minus that;
 *   - softened and truncated force = spline force x short-range factor;
 *   - fourth-order four-point finite differences; deconvolution by
 *     sinc^2 (assignment) x sinc^2 (interpolation) per axis;
 *   - isolated mesh: ng cells of h = L_root / (ng - 4) cover the root cube
 *     with two spare cells per side, zero-padded to (2 ng)^3, r_s = asmth h;
 *   - individual softening: spline supports 2.8 eps_i, a pair uses the larger,
 *     a node carries the largest of its particles and, when that exceeds the
 *     target's, is opened for distances to its centre of mass below it and
 *     otherwise interacts with the larger of the target's and its own.
 *
 * Floating point: compiled with -ffp-contract=off; fused multiply-adds are
 * written explicitly with fma() where the arithmetic contract uses them.
 *
 * Mutation builds (-DORC_MUTATION=k) plant one deliberate mistake each so
 * the tests can show that their pins catch it; the normal build uses 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_BITS 21
#define ORC_MAXLEVEL 21

#ifndef ORC_MUTATION
#define ORC_MUTATION 0
#endif

/* ------------------------------------------------------------------ */
/* Peano-Hilbert key (Sec. 8: domain pieces are Peano-Hilbert          */
/* adjacent).  Skilling, "Programming the Hilbert curve", AIP Conf.    */
/* Proc. 707 (2004): axes -> transpose form, then bit interleave.      */
/* ------------------------------------------------------------------ */
uint64_t orc_ph_key(int b, uint32_t c0, uint32_t c1, uint32_t c2)
{
    uint32_t X[3];
    X[0] = c0;
    X[1] = c1;
    X[2] = c2;
    uint32_t M = 1u << (b - 1);
    /* undo excess work, from the top bit down: invert or exchange */
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        uint32_t P = Q - 1;
        for (int i = 0; i < 3; i++) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    /* Gray encode */
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q)
            t ^= Q - 1;
#if ORC_MUTATION != 8
    for (int i = 0; i < 3; i++)
        X[i] ^= t;
#endif
    /* transpose -> key: bit j of X0, X1, X2 from the top bit down */
    uint64_t h = 0;
    for (int j = b - 1; j >= 0; j--) {
        h = (h << 3) | ((uint64_t)((X[0] >> j) & 1u) << 2) |
            ((uint64_t)((X[1] >> j) & 1u) << 1) | (uint64_t)((X[2] >> j) & 1u);
    }
    return h;
}

void orc_ph_keys_b(int b, int64_t n, const uint32_t *q0, const uint32_t *q1,
                   const uint32_t *q2, uint64_t *key)
{
    for (int64_t i = 0; i < n; i++)
        key[i] = orc_ph_key(b, q0[i], q1[i], q2[i]);
}

/* ------------------------------------------------------------------ */
/* Root cube (Sec. 3.1: an all-enclosing cubical root node; random     */
/* placement of the tree domain / random shift of a periodic box).     */
/* frame = {x0, y0, z0, L_root}; shift[a] in [0,1) is passed in.       */
/* ------------------------------------------------------------------ */
void orc_frame(int64_t n, const double *x, const double *y, const double *z,
               int periodic, double box, const double *shift, double *frame)
{
    const double *c[3] = {x, y, z};
    if (periodic) {
        for (int a = 0; a < 3; a++)
            frame[a] = -(shift[a] * box);
        frame[3] = box;
        return;
    }
    double lo[3], hi[3], ext = 0.0;
    for (int a = 0; a < 3; a++) {
        lo[a] = c[a][0];
        hi[a] = c[a][0];
        for (int64_t i = 1; i < n; i++) {
            if (c[a][i] < lo[a])
                lo[a] = c[a][i];
            if (c[a][i] > hi[a])
                hi[a] = c[a][i];
        }
        double e = hi[a] - lo[a];
        if (e > ext)
            ext = e;
    }
    /* smallest power of two >= ext * (1 + 2^-20); 1 if all coincide */
    double L = 1.0;
    if (ext > 0.0) {
        double target = ext * (1.0 + 0x1p-20);
        int e2;
        double m = frexp(target, &e2);
        L = (m == 0.5) ? ldexp(1.0, e2 - 1) : ldexp(1.0, e2);
    }
    for (int a = 0; a < 3; a++) {
        double slack = L - (hi[a] - lo[a]);
        frame[a] = lo[a] - shift[a] * slack;
    }
    frame[3] = L;
}

/* Tree-frame coordinate p (periodic: moved by one box length into
 * [x0, x0 + L)) and its 21-bit integer coordinate q. */
static void frame_coord(double xv, double x0, double L, int periodic, double *p_out,
                        uint32_t *q_out)
{
    double p = xv;
    double u = p - x0;
    if (periodic) {
        if (u >= L) {
            p = xv - L;
            u = p - x0;
        } else if (u < 0.0) {
            p = xv + L;
            u = p - x0;
        }
    }
    double S = 2097152.0 / L; /* 2^21 / L_root */
    double f = floor(u * S);
    if (f < 0.0)
        f = 0.0;
    if (f > 2097151.0)
        f = 2097151.0;
    *p_out = p;
    *q_out = (uint32_t)f;
}

void orc_positions(int64_t n, const double *x, const double *y, const double *z,
                   int periodic, const double *frame, double *p /* 3n or NULL */,
                   uint32_t *q /* 3n or NULL */, uint64_t *key /* n or NULL */)
{
    const double *c[3] = {x, y, z};
    for (int64_t i = 0; i < n; i++) {
        double pp[3];
        uint32_t qq[3];
        for (int a = 0; a < 3; a++)
            frame_coord(c[a][i], frame[a], frame[3], periodic, &pp[a], &qq[a]);
        for (int a = 0; a < 3; a++) {
            if (p)
                p[a * n + i] = pp[a];
            if (q)
                q[a * n + i] = qq[a];
        }
        if (key)
            key[i] = orc_ph_key(ORC_BITS, qq[0], qq[1], qq[2]);
    }
}

/* Ascending sort of particle indices by key, ties by index. */
static const uint64_t *g_sort_keys;
static int cmp_key_idx(const void *A, const void *B)
{
    int64_t a = *(const int64_t *)A, b = *(const int64_t *)B;
    if (g_sort_keys[a] < g_sort_keys[b])
        return -1;
    if (g_sort_keys[a] > g_sort_keys[b])
        return 1;
    return (a < b) ? -1 : (a > b);
}

void orc_sort(int64_t n, const uint64_t *key, int64_t *perm)
{
    for (int64_t i = 0; i < n; i++)
        perm[i] = i;
    g_sort_keys = key;
    qsort(perm, (size_t)n, sizeof(int64_t), cmp_key_idx);
    g_sort_keys = NULL;
}

/* ------------------------------------------------------------------ */
/* Octree by sequential insertion (Sec. 3.1): a leaf that receives a   */
/* second particle is split and its resident moved down, until every   */
/* leaf holds one particle; depth-21 cells keep a list instead.        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t child[8];
    int64_t head; /* leaf: first particle of its list; -1 when internal */
    int level;
    uint32_t corner[3]; /* integer corner, in cells of its own level */
    int is_leaf;
} inode;

typedef struct orc_tree {
    int64_t n;
    int periodic;
    double frame[4];
    double *p;    /* 3n tree-frame positions [a*n + i] */
    uint32_t *q;  /* 3n integer coordinates */
    uint64_t *key;
    double *mass; /* n */
    inode *nodes;
    int64_t nnodes, cap;
    int64_t *next_in_leaf;
    int32_t root;
    /* canonical depth-first entry list (nodes and particles) */
    int64_t E, Ecap;
    int32_t *level; /* -1 marks a particle entry */
    int64_t *first, *count, *skip, *pidx;
    double *emass, *com, *cen; /* com, cen: [a*Ecap + e] */
    int64_t *entry_of; /* particle index -> its entry */
    int64_t nemitted;  /* particles emitted so far */
    /* individual softening (Sec. 3.2), NULL when all particles share eps:
     * hsoft[i] = 2.8 eps_i, eh[e] = largest hsoft in entry e */
    double *hsoft, *eh;
} orc_tree;

static int32_t new_inode(orc_tree *T, int level, const uint32_t corner[3])
{
    if (T->nnodes == T->cap) {
        T->cap = T->cap ? 2 * T->cap : 1024;
        T->nodes = (inode *)realloc(T->nodes, (size_t)T->cap * sizeof(inode));
    }
    inode *nd = &T->nodes[T->nnodes];
    for (int k = 0; k < 8; k++)
        nd->child[k] = -1;
    nd->head = -1;
    nd->level = level;
    nd->is_leaf = 1;
    for (int a = 0; a < 3; a++)
        nd->corner[a] = corner[a];
    return (int32_t)T->nnodes++;
}

/* child slot and child corner of particle i below a node of level lev */
static int child_of(const orc_tree *T, int64_t i, int lev, const uint32_t parent[3],
                    uint32_t out[3])
{
    int bit = ORC_BITS - 1 - lev;
    int o = 0;
    for (int a = 0; a < 3; a++) {
        uint32_t b = (T->q[a * T->n + i] >> bit) & 1u;
        o |= (int)b << (2 - a);
        out[a] = 2u * parent[a] + b;
    }
    return o;
}

static void tree_insert(orc_tree *T, int64_t i)
{
    uint32_t cc[3], par[3];
    T->next_in_leaf[i] = -1;
    if (T->root < 0) {
        uint32_t z3[3] = {0, 0, 0};
        T->root = new_inode(T, 0, z3);
        T->nodes[T->root].head = i;
        return;
    }
    int32_t nd = T->root;
    for (;;) {
        int lev = T->nodes[nd].level;
        memcpy(par, T->nodes[nd].corner, sizeof par);
        if (!T->nodes[nd].is_leaf) {
            int o = child_of(T, i, lev, par, cc);
            int32_t c = T->nodes[nd].child[o];
            if (c < 0) {
                c = new_inode(T, lev + 1, cc);
                T->nodes[c].head = i;
                T->nodes[nd].child[o] = c;
                return;
            }
            nd = c;
            continue;
        }
        if (lev == ORC_MAXLEVEL) { /* depth limit: append to the cell's list */
            int64_t j = T->nodes[nd].head;
            while (T->next_in_leaf[j] >= 0)
                j = T->next_in_leaf[j];
            T->next_in_leaf[j] = i;
            return;
        }
        /* occupied leaf: split it and move its resident particle down */
        int64_t j = T->nodes[nd].head;
        int o = child_of(T, j, lev, par, cc);
        int32_t c = new_inode(T, lev + 1, cc);
        T->nodes[c].head = j;
        T->nodes[nd].is_leaf = 0;
        T->nodes[nd].head = -1;
        T->nodes[nd].child[o] = c;
        /* and try again with particle i at the now internal node */
    }
}

static uint64_t subtree_min_key(const orc_tree *T, int32_t nd)
{
    const inode *N = &T->nodes[nd];
    uint64_t m = UINT64_MAX;
    if (N->is_leaf) {
        for (int64_t j = N->head; j >= 0; j = T->next_in_leaf[j])
            if (T->key[j] < m)
                m = T->key[j];
        return m;
    }
    for (int k = 0; k < 8; k++)
        if (N->child[k] >= 0) {
            uint64_t c = subtree_min_key(T, N->child[k]);
            if (c < m)
                m = c;
        }
    return m;
}

static int64_t add_entry(orc_tree *T, int level, int64_t pidx)
{
    int64_t e = T->E++;
    T->level[e] = level;
    T->pidx[e] = pidx;
    T->first[e] = T->nemitted;
    T->count[e] = 0;
    T->skip[e] = e + 1;
    return e;
}

static void set_node_geometry(orc_tree *T, int64_t e, int level, const uint32_t corner[3])
{
    double len = ldexp(T->frame[3], -level);
    for (int a = 0; a < 3; a++)
        T->cen[a * T->Ecap + e] = T->frame[a] + ((double)corner[a] + 0.5) * len;
}

static void emit_particle(orc_tree *T, int64_t i)
{
    int64_t e = add_entry(T, -1, i);
    T->count[e] = 1;
    T->emass[e] = T->mass[i];
    for (int a = 0; a < 3; a++) {
        T->com[a * T->Ecap + e] = T->p[a * T->n + i];
        T->cen[a * T->Ecap + e] = T->p[a * T->n + i];
    }
    T->entry_of[i] = e;
    T->nemitted++;
}

/* Monopole moments of node e from its children, in curve order (Sec. 3.1):
 * M = (M1 + M2) + ...,  X_a = fma(Mk, s_k,a, X_a),  s_a = X_a / M. */
static void node_moments(orc_tree *T, int64_t e)
{
    double M = 0.0, X[3] = {0.0, 0.0, 0.0};
    for (int64_t k = e + 1; k < T->skip[e]; k = T->skip[k]) {
        double mk = T->emass[k];
        M = M + mk;
        for (int a = 0; a < 3; a++)
            X[a] = fma(mk, T->com[a * T->Ecap + k], X[a]);
    }
    T->emass[e] = M;
    for (int a = 0; a < 3; a++)
#if ORC_MUTATION == 5
        T->com[a * T->Ecap + e] = X[a];
#else
        T->com[a * T->Ecap + e] = X[a] / M;
#endif
}

static int cmp_i64(const void *A, const void *B)
{
    int64_t a = *(const int64_t *)A, b = *(const int64_t *)B;
    return (a > b) - (a < b);
}

static void emit(orc_tree *T, int32_t nd)
{
    const inode *N = &T->nodes[nd];
    if (N->is_leaf) {
        int64_t cnt = 0;
        for (int64_t j = N->head; j >= 0; j = T->next_in_leaf[j])
            cnt++;
        if (cnt == 1) {
            emit_particle(T, N->head);
            return;
        }
        /* depth-21 cell with several particles: a node entry, then its
         * particles ordered by index */
        int64_t *lst = (int64_t *)malloc((size_t)cnt * sizeof(int64_t));
        int64_t c = 0;
        for (int64_t j = N->head; j >= 0; j = T->next_in_leaf[j])
            lst[c++] = j;
        qsort(lst, (size_t)cnt, sizeof(int64_t), cmp_i64);
        int64_t e = add_entry(T, N->level, -1);
        set_node_geometry(T, e, N->level, N->corner);
        for (int64_t k = 0; k < cnt; k++)
            emit_particle(T, lst[k]);
        free(lst);
        T->skip[e] = T->E;
        T->count[e] = T->nemitted - T->first[e];
        node_moments(T, e);
        return;
    }
    int64_t e = add_entry(T, N->level, -1);
    set_node_geometry(T, e, N->level, N->corner);
    /* children in Peano-Hilbert order: by the smallest key they hold */
    int32_t ch[8];
    uint64_t mk[8];
    int nc = 0;
    for (int k = 0; k < 8; k++)
        if (N->child[k] >= 0) {
            ch[nc] = N->child[k];
            mk[nc] = subtree_min_key(T, N->child[k]);
            nc++;
        }
    for (int a = 1; a < nc; a++) /* insertion sort of at most 8 */
        for (int b = a; b > 0 && mk[b] < mk[b - 1]; b--) {
            uint64_t t = mk[b];
            mk[b] = mk[b - 1];
            mk[b - 1] = t;
            int32_t c = ch[b];
            ch[b] = ch[b - 1];
            ch[b - 1] = c;
        }
    for (int k = 0; k < nc; k++)
        emit(T, ch[k]);
    T->skip[e] = T->E;
    T->count[e] = T->nemitted - T->first[e];
    node_moments(T, e);
}

orc_tree *orc_tree_build(int64_t n, const double *x, const double *y, const double *z,
                         const double *mass, int periodic, double box,
                         const double *shift, const int64_t *insert_order)
{
    orc_tree *T = (orc_tree *)calloc(1, sizeof(orc_tree));
    T->n = n;
    T->periodic = periodic;
    orc_frame(n, x, y, z, periodic, box, shift, T->frame);
    T->p = (double *)malloc((size_t)(3 * n) * sizeof(double));
    T->q = (uint32_t *)malloc((size_t)(3 * n) * sizeof(uint32_t));
    T->key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    T->mass = (double *)malloc((size_t)n * sizeof(double));
    orc_positions(n, x, y, z, periodic, T->frame, T->p, T->q, T->key);
    for (int64_t i = 0; i < n; i++)
        T->mass[i] = mass ? mass[i] : 1.0 / (double)n;
    T->next_in_leaf = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    T->root = -1;
    for (int64_t k = 0; k < n; k++)
        tree_insert(T, insert_order ? insert_order[k] : k);
    T->Ecap = T->nnodes + n;
    T->level = (int32_t *)malloc((size_t)T->Ecap * sizeof(int32_t));
    T->first = (int64_t *)malloc((size_t)T->Ecap * sizeof(int64_t));
    T->count = (int64_t *)malloc((size_t)T->Ecap * sizeof(int64_t));
    T->skip = (int64_t *)malloc((size_t)T->Ecap * sizeof(int64_t));
    T->pidx = (int64_t *)malloc((size_t)T->Ecap * sizeof(int64_t));
    T->emass = (double *)malloc((size_t)T->Ecap * sizeof(double));
    T->com = (double *)malloc((size_t)(3 * T->Ecap) * sizeof(double));
    T->cen = (double *)malloc((size_t)(3 * T->Ecap) * sizeof(double));
    T->entry_of = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    T->E = 0;
    T->nemitted = 0;
    emit(T, T->root);
    return T;
}

int64_t orc_tree_entries(const orc_tree *T) { return T->E; }

void orc_tree_frame(const orc_tree *T, double *frame)
{
    memcpy(frame, T->frame, 4 * sizeof(double));
}

/* Copy the depth-first list out (any pointer may be NULL). */
void orc_tree_export(const orc_tree *T, int32_t *level, int64_t *first, int64_t *count,
                     int64_t *skip, int64_t *pidx, double *mass, double *com,
                     double *cen)
{
    int64_t E = T->E;
    for (int64_t e = 0; e < E; e++) {
        if (level)
            level[e] = T->level[e];
        if (first)
            first[e] = T->first[e];
        if (count)
            count[e] = T->count[e];
        if (skip)
            skip[e] = T->skip[e];
        if (pidx)
            pidx[e] = T->pidx[e];
        if (mass)
            mass[e] = T->emass[e];
        for (int a = 0; a < 3; a++) {
            if (com)
                com[a * E + e] = T->com[a * T->Ecap + e];
            if (cen)
                cen[a * E + e] = T->cen[a * T->Ecap + e];
        }
    }
}

void orc_tree_positions(const orc_tree *T, double *p, uint32_t *q, uint64_t *key)
{
    int64_t n = T->n;
    if (p)
        memcpy(p, T->p, (size_t)(3 * n) * sizeof(double));
    if (q)
        memcpy(q, T->q, (size_t)(3 * n) * sizeof(uint32_t));
    if (key)
        memcpy(key, T->key, (size_t)n * sizeof(uint64_t));
}

/* Individual softening lengths (Sec. 3.2): each entry carries the largest
 * spline support of the particles it holds (a particle its own). */
void orc_tree_set_softening(orc_tree *T, const double *eps)
{
    free(T->hsoft);
    free(T->eh);
    T->hsoft = (double *)malloc((size_t)T->n * sizeof(double));
    T->eh = (double *)malloc((size_t)T->E * sizeof(double));
    for (int64_t i = 0; i < T->n; i++)
        T->hsoft[i] = 2.8 * eps[i];
    for (int64_t e = T->E - 1; e >= 0; e--) { /* children follow their node */
        if (T->level[e] < 0) {
            T->eh[e] = T->hsoft[T->pidx[e]];
            continue;
        }
        double m = 0.0;
        for (int64_t k = e + 1; k < T->skip[e]; k = T->skip[k])
            m = T->eh[k] > m ? T->eh[k] : m;
        T->eh[e] = m;
    }
}

void orc_tree_free(orc_tree *T)
{
    if (!T)
        return;
    free(T->hsoft);
    free(T->eh);
    free(T->p);
    free(T->q);
    free(T->key);
    free(T->mass);
    free(T->nodes);
    free(T->next_in_leaf);
    free(T->level);
    free(T->first);
    free(T->count);
    free(T->skip);
    free(T->pidx);
    free(T->emass);
    free(T->com);
    free(T->cen);
    free(T->entry_of);
    free(T);
}

/* ------------------------------------------------------------------ */
/* Interaction kernels                                                 */
/* ------------------------------------------------------------------ */
typedef struct orc_params {
    int periodic;
    int opening;   /* 0: geometric (Barnes-Hut), 1: relative */
    int treepm;    /* short-range truncation and cutoff on */
    int want_pot;
    double box;
    double G;
    double eps;    /* Plummer-equivalent softening; spline support 2.8 eps */
    double theta;
    double alpha;
    double rs;     /* split scale */
    double rcut;   /* cutoff radius (absolute) */
} orc_params;

/* Spline-softened force factor g(u) for u < 1, with r-vector force
 * a = G m g(u) / h^3 * d  (Sec. 3.2; cubic spline kernel, support h). */
static double spline_g(double u)
{
    if (u < 0.5) {
        double u2 = u * u;
        return fma(u2, fma(32.0, u, -38.4), 32.0 / 3.0);
    }
    double cubic = fma(fma(fma(-32.0 / 3.0, u, 38.4), u, -48.0), u, 64.0 / 3.0);
    return cubic - 1.0 / (15.0 * (u * u * u));
}

/* Spline-softened potential phi(u) * (h / G m) for u < 1 (phi(0)*h/Gm = -14/5). */
static double spline_phi(double u)
{
    double u2 = u * u;
    if (u < 0.5)
        return u2 * (16.0 / 3.0 + u2 * (-48.0 / 5.0 + u * (32.0 / 5.0))) - 14.0 / 5.0;
    return u2 * (32.0 / 3.0 + u * (-16.0 + u * (48.0 / 5.0 + u * (-32.0 / 15.0)))) -
           16.0 / 5.0 + 1.0 / (15.0 * u);
}

static const double TWO_OVER_SQRTPI = 1.1283791670955126;

/* Short-range force factor f_s(r) (Sec. 3.4, sign of the exponent read as
 * negative and the factor read as the short-range one). */
static double short_range_factor(double r, double rs)
{
    double x = r * (0.5 / rs);
#if ORC_MUTATION == 3
    return erfc(x);
#else
    return erfc(x) + (x * TWO_OVER_SQRTPI) * exp(-(x * x));
#endif
}

/* add the interaction of mass m at offset d (target -> source) */
static void interact(const orc_params *P, double h, double hinv, double h3inv, double m,
                     const double d[3], double d2, double acc[3], double *pot)
{
    double Gm = P->G * m;
#if ORC_MUTATION == 1
    Gm = Gm * 1.01;
#endif
    double r = sqrt(d2);
    double fac, phi = 0.0;
    if (r >= h) {
        double rinv = 1.0 / r;
        fac = Gm * rinv * rinv * rinv;
        if (P->want_pot)
            phi = -Gm * rinv;
    } else {
        double u = r / h;
        fac = (Gm * h3inv) * spline_g(u);
        if (P->want_pot)
            phi = (Gm * hinv) * spline_phi(u);
    }
    if (P->treepm) {
        fac = fac * short_range_factor(r, P->rs);
        if (P->want_pot)
            phi = phi * erfc(r * (0.5 / P->rs));
    }
    for (int a = 0; a < 3; a++)
        acc[a] = fma(fac, d[a], acc[a]);
    if (P->want_pot)
        *pot += phi;
}

static double wrap(const orc_params *P, double d)
{
    if (!P->periodic)
        return d;
    double half = 0.5 * P->box;
#if ORC_MUTATION == 4
    if (d > half)
        d += P->box;
    else if (d < -half)
        d -= P->box;
#else
    if (d > half)
        d -= P->box;
    else if (d < -half)
        d += P->box;
#endif
    return d;
}

/* ------------------------------------------------------------------ */
/* Tree walk for one target (Sec. 3.1 opening criteria, Sec. 3.4 cut). */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_tree *T;
    const orc_params *P;
    int64_t self;
    double x[3];
    double anorm;
    double h, hinv, h3inv, rc2;
    double hself; /* the target's own spline support */
    double acc[3];
    double pot;
    int64_t nint;
} walk_state;

static void visit(walk_state *W, int64_t e)
{
    const orc_tree *T = W->T;
    const orc_params *P = W->P;
    int64_t Ec = T->Ecap;
    double d[3];
    for (int a = 0; a < 3; a++)
        d[a] = wrap(P, T->com[a * Ec + e] - W->x[a]);
    double d2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
    if (T->level[e] < 0) { /* particle */
        if (T->pidx[e] == W->self)
            return;
        if (P->treepm && !(d2 < W->rc2))
            return;
        if (T->eh) { /* pair softening: the larger of the two (Sec. 3.2) */
#if ORC_MUTATION == 12
            double h = W->hself;
#else
            double h = W->hself > T->eh[e] ? W->hself : T->eh[e];
#endif
            double hinv = 1.0 / h;
            interact(P, h, hinv, hinv * hinv * hinv, T->emass[e], d, d2, W->acc, &W->pot);
        } else {
            interact(P, W->h, W->hinv, W->h3inv, T->emass[e], d, d2, W->acc, &W->pot);
        }
        W->nint++;
        return;
    }
    double L = ldexp(T->frame[3], -T->level[e]);
    double dc[3];
    for (int a = 0; a < 3; a++)
        dc[a] = wrap(P, T->cen[a * Ec + e] - W->x[a]);
    if (P->treepm) { /* discard a cube that lies wholly beyond the cutoff */
        double ex[3];
        for (int a = 0; a < 3; a++) {
            double t = fabs(dc[a]) - 0.5 * L;
            ex[a] = t > 0.0 ? t : 0.0;
        }
        double s2 = fma(ex[0], ex[0], fma(ex[1], ex[1], ex[2] * ex[2]));
        if (s2 > W->rc2)
            return;
    }
    int open;
    if (P->opening == 0) {
#if ORC_MUTATION == 9
        open = (L * L) > P->theta * d2;
#else
        open = (L * L) > (P->theta * P->theta) * d2;
#endif
    } else {
#if ORC_MUTATION == 14
        open = (L * L) > (P->alpha * W->anorm) * (d2 * d2);
#elif ORC_MUTATION == 15
        open = (P->G * T->emass[e]) * L > (P->alpha * W->anorm) * (d2 * d2);
#elif ORC_MUTATION == 16
        open = (P->G * T->emass[e]) * (L * L) > P->alpha * (d2 * d2);
#elif ORC_MUTATION == 17
        open = (P->G * T->emass[e]) * (L * L) > (P->alpha * W->anorm) * d2;
#else
        open = (P->G * T->emass[e]) * (L * L) > (P->alpha * W->anorm) * (d2 * d2);
#endif
    }
    /* 1.2 L box around the geometric centre: always open */
    double lim = 0.6 * L;
#if ORC_MUTATION != 2
    if (fabs(dc[0]) < lim && fabs(dc[1]) < lim && fabs(dc[2]) < lim)
        open = 1;
#endif
    /* a node holding larger softenings than the target's is opened when the
     * target lies within that softening of its centre of mass (Sec. 3.2) */
#if ORC_MUTATION != 13
    if (T->eh && W->hself < T->eh[e] && d2 < T->eh[e] * T->eh[e])
        open = 1;
#endif
    if (open) {
        for (int64_t k = e + 1; k < T->skip[e]; k = T->skip[k])
            visit(W, k);
        return;
    }
    if (T->eh) {
        double h = W->hself > T->eh[e] ? W->hself : T->eh[e];
        double hinv = 1.0 / h;
        interact(P, h, hinv, hinv * hinv * hinv, T->emass[e], d, d2, W->acc, &W->pot);
    } else {
        interact(P, W->h, W->hinv, W->h3inv, T->emass[e], d, d2, W->acc, &W->pot);
    }
    W->nint++;
}

/* acc: [3][nt]; pot: nt or NULL; nint: nt or NULL; anorm by particle index
 * (NULL only for the geometric criterion). */
void orc_tree_walk(const orc_tree *T, const orc_params *P, int64_t nt,
                   const int64_t *targets, const double *anorm, double *acc, double *pot,
                   int64_t *nint)
{
    double h = 2.8 * P->eps;
    double hinv = 1.0 / h;
    double h3inv = hinv * hinv * hinv;
    double rc2 = P->rcut * P->rcut;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; k++) {
        walk_state W;
        int64_t i = targets[k];
        W.T = T;
        W.P = P;
        W.self = i;
        for (int a = 0; a < 3; a++)
            W.x[a] = T->p[a * T->n + i];
        W.anorm = anorm ? anorm[i] : 0.0;
        W.h = h;
        W.hinv = hinv;
        W.h3inv = h3inv;
        W.hself = T->hsoft ? T->hsoft[i] : h;
        W.rc2 = rc2;
        W.acc[0] = W.acc[1] = W.acc[2] = 0.0;
        W.pot = 0.0;
        W.nint = 0;
        visit(&W, 0);
        for (int a = 0; a < 3; a++)
            acc[a * nt + k] = W.acc[a];
        if (pot)
            pot[k] = W.pot;
        if (nint)
            nint[k] = W.nint;
    }
}

/* ------------------------------------------------------------------ */
/* Direct summation (the exact reference, Sec. 3 introduction): every  */
/* pair, spline softening; with TreePM only the truncated short-range  */
/* part of the nearest image inside the cutoff.                        */
/* ------------------------------------------------------------------ */
void orc_direct(int64_t n, const double *x, const double *y, const double *z,
                const double *mass, const double *eps /* per particle or NULL */,
                const orc_params *P, int64_t nt, const int64_t *targets, double *acc,
                double *pot)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; k++) {
        int64_t i = targets[k];
        double a[3] = {0, 0, 0}, ph = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i)
                continue;
            double d[3] = {x[j] - x[i], y[j] - y[i], z[j] - z[i]};
            if (P->periodic)
                for (int c = 0; c < 3; c++)
                    d[c] -= P->box * nearbyint(d[c] / P->box);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (P->treepm && r >= P->rcut)
                continue;
            double m = mass ? mass[j] : 1.0 / (double)n;
            /* individual softening: symmetrised by the larger one (Sec. 3.2) */
            double h = 2.8 * (eps ? (eps[i] > eps[j] ? eps[i] : eps[j]) : P->eps);
            double f, phi;
            double u = r / h;
            if (u >= 1.0) {
                f = P->G * m / (r * r * r);
                phi = -P->G * m / r;
            } else if (u < 0.5) {
                f = P->G * m / (h * h * h) * (32.0 / 3.0 - 192.0 / 5.0 * u * u + 32.0 * u * u * u);
                phi = P->G * m / h *
                      (16.0 / 3.0 * u * u - 48.0 / 5.0 * pow(u, 4) + 32.0 / 5.0 * pow(u, 5) -
                       14.0 / 5.0);
            } else {
                f = P->G * m / (h * h * h) *
                    (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u * u - 32.0 / 3.0 * u * u * u -
                     1.0 / (15.0 * u * u * u));
                phi = P->G * m / h *
                      (32.0 / 3.0 * u * u - 16.0 * u * u * u + 48.0 / 5.0 * pow(u, 4) -
                       32.0 / 15.0 * pow(u, 5) - 16.0 / 5.0 + 1.0 / (15.0 * u));
            }
            if (P->treepm) {
                double s = r / (2.0 * P->rs);
                f *= erfc(s) + 2.0 * s / sqrt(M_PI) * exp(-s * s);
                phi *= erfc(s);
            }
            for (int c = 0; c < 3; c++)
                a[c] += f * d[c];
            ph += phi;
        }
        for (int c = 0; c < 3; c++)
            acc[c * nt + k] = a[c];
        if (pot)
            pot[k] = ph;
    }
}

/* ------------------------------------------------------------------ */
/* Textbook FFT: iterative radix-2 Cooley-Tukey on one complex line.   */
/* sign = -1 forward, +1 inverse (unnormalised).                       */
/* ------------------------------------------------------------------ */
static void fft_line(int n, double *re, double *im, int sign, const double *wr,
                     const double *wi)
{
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i];
            re[i] = re[j];
            re[j] = t;
            t = im[i];
            im[i] = im[j];
            im[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len >> 1, step = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < half; k++) {
#if ORC_MUTATION == 6
                double cr = wr[k * step], ci = -sign * wi[k * step];
#else
                double cr = wr[k * step], ci = sign * wi[k * step];
#endif
                double vr = re[i + k + half] * cr - im[i + k + half] * ci;
                double vi = re[i + k + half] * ci + im[i + k + half] * cr;
                re[i + k + half] = re[i + k] - vr;
                im[i + k + half] = im[i + k] - vi;
                re[i + k] += vr;
                im[i + k] += vi;
            }
    }
}

/* In-place 3-D complex FFT of an n^3 array (index (i*n + j)*n + k). */
void orc_fft3(int n, double *re, double *im, int sign)
{
    double *wr = (double *)malloc((size_t)n * sizeof(double));
    double *wi = (double *)malloc((size_t)n * sizeof(double));
    for (int k = 0; k < n; k++) { /* twiddle exp(sign * 2 pi i k / n) = wr + i sign wi */
        wr[k] = cos(2.0 * M_PI * k / n);
        wi[k] = sin(2.0 * M_PI * k / n);
    }
    double *lr = (double *)malloc((size_t)n * sizeof(double));
    double *li = (double *)malloc((size_t)n * sizeof(double));
    int64_t n2 = (int64_t)n * n;
    for (int axis = 0; axis < 3; axis++) {
        int64_t stride = axis == 0 ? n2 : (axis == 1 ? n : 1);
        for (int64_t a = 0; a < n; a++)
            for (int64_t b = 0; b < n; b++) {
                int64_t base;
                if (axis == 0)
                    base = a * n + b;
                else if (axis == 1)
                    base = a * n2 + b;
                else
                    base = a * n2 + b * n;
                for (int k = 0; k < n; k++) {
                    lr[k] = re[base + k * stride];
                    li[k] = im[base + k * stride];
                }
                fft_line(n, lr, li, sign, wr, wi);
                for (int k = 0; k < n; k++) {
                    re[base + k * stride] = lr[k];
                    im[base + k * stride] = li[k];
                }
            }
    }
    free(wr);
    free(wi);
    free(lr);
    free(li);
}

/* ------------------------------------------------------------------ */
/* Particle-mesh long-range force (Sec. 3.3, 3.4).                     */
/* ------------------------------------------------------------------ */

/* Mesh part: density rho (ng^3, mass per unit volume) -> potential and
 * the three force meshes.  Phi_k = -4 pi G rho_k exp(-k^2 rs^2) /
 * (k^2 prod_a sinc^4(k_a h / 2)), k = 0 removed (mean density subtracted,
 * Sec. 2.2), Phi = IFFT / ng^3; a = -grad Phi by four-point differences. */
void orc_pm_mesh(int ng, double box, double G, double rs, const double *rho,
                 double *phi /* ng^3 */, double *fx, double *fy, double *fz)
{
    int64_t n3 = (int64_t)ng * ng * ng;
    double *re = (double *)malloc((size_t)n3 * sizeof(double));
    double *im = (double *)calloc((size_t)n3, sizeof(double));
    memcpy(re, rho, (size_t)n3 * sizeof(double));
    orc_fft3(ng, re, im, -1);
    double h = box / ng;
    for (int i = 0; i < ng; i++)
        for (int j = 0; j < ng; j++)
            for (int k = 0; k < ng; k++) {
                int64_t c = ((int64_t)i * ng + j) * ng + k;
                int n[3] = {i < ng / 2 ? i : i - ng, j < ng / 2 ? j : j - ng,
                            k < ng / 2 ? k : k - ng};
                double kv[3], k2 = 0.0, deconv = 1.0;
                for (int a = 0; a < 3; a++) {
                    kv[a] = 2.0 * M_PI * n[a] / box;
                    k2 += kv[a] * kv[a];
                    double s = 0.5 * kv[a] * h;
                    double sc = (n[a] == 0) ? 1.0 : sin(s) / s;
                    deconv *= sc * sc * sc * sc;
                }
                double g;
                if (k2 == 0.0)
                    g = 0.0;
                else
                    g = -4.0 * M_PI * G * exp(-k2 * rs * rs) / (k2 * deconv);
                re[c] *= g;
                im[c] *= g;
            }
    orc_fft3(ng, re, im, +1);
    for (int64_t c = 0; c < n3; c++)
        phi[c] = re[c] / (double)n3;
    free(re);
    free(im);
    double *F[3] = {fx, fy, fz};
    for (int i = 0; i < ng; i++)
        for (int j = 0; j < ng; j++)
            for (int k = 0; k < ng; k++) {
                int idx[3] = {i, j, k};
                for (int a = 0; a < 3; a++) {
                    double v[5];
                    for (int s = -2; s <= 2; s++) {
                        int t[3] = {idx[0], idx[1], idx[2]};
                        t[a] = ((t[a] + s) % ng + ng) % ng;
                        v[s + 2] = phi[((int64_t)t[0] * ng + t[1]) * ng + t[2]];
                    }
#if ORC_MUTATION == 7
                    double grad = ((2.0 / 3.0) * (v[3] - v[1]) - (1.0 / 6.0) * (v[4] - v[0])) / h;
#else
                    double grad = ((2.0 / 3.0) * (v[3] - v[1]) - (1.0 / 12.0) * (v[4] - v[0])) / h;
#endif
                    F[a][((int64_t)i * ng + j) * ng + k] = -grad;
                }
            }
}

/* CIC weights of one position: base cell and weight of the upper cell. */
static void cic_weights(double pos, double box, int ng, int *i0, double *w)
{
    double u = pos;
    if (u < 0.0)
        u += box;
    if (u >= box)
        u -= box;
    double f = u / (box / ng);
    double fl = floor(f);
#if ORC_MUTATION == 10
    *w = 1.0 - (f - fl);
#else
    *w = f - fl;
#endif
    int i = (int)fl;
    if (i >= ng)
        i -= ng;
    if (i < 0)
        i += ng;
    *i0 = i;
}

void orc_cic_deposit(int64_t n, const double *x, const double *y, const double *z,
                     const double *mass, double box, int ng, double *rho)
{
    int64_t n3 = (int64_t)ng * ng * ng;
    double h = box / ng;
    double vinv = 1.0 / (h * h * h);
    memset(rho, 0, (size_t)n3 * sizeof(double));
    const double *c[3] = {x, y, z};
    for (int64_t p = 0; p < n; p++) {
        int i0[3];
        double w[3];
        for (int a = 0; a < 3; a++)
            cic_weights(c[a][p], box, ng, &i0[a], &w[a]);
        double m = mass ? mass[p] : 1.0 / (double)n;
        for (int s = 0; s < 8; s++) {
            double wt = 1.0;
            int t[3];
            for (int a = 0; a < 3; a++) {
                int up = (s >> (2 - a)) & 1;
                wt *= up ? w[a] : 1.0 - w[a];
                t[a] = up ? (i0[a] + 1) % ng : i0[a];
            }
            rho[((int64_t)t[0] * ng + t[1]) * ng + t[2]] += m * wt * vinv;
        }
    }
}

static double cic_interp(const double *mesh, int ng, const int i0[3], const double w[3])
{
    double v = 0.0;
    for (int s = 0; s < 8; s++) {
        double wt = 1.0;
        int t[3];
        for (int a = 0; a < 3; a++) {
            int up = (s >> (2 - a)) & 1;
            wt *= up ? w[a] : 1.0 - w[a];
            t[a] = up ? (i0[a] + 1) % ng : i0[a];
        }
        v += wt * mesh[((int64_t)t[0] * ng + t[1]) * ng + t[2]];
    }
    return v;
}

/* Full PM long-range force at the targets: deposit all particles, solve,
 * difference, interpolate.  acc [3][nt]; pot nt or NULL. */
void orc_pm(int64_t n, const double *x, const double *y, const double *z,
            const double *mass, double box, int ng, double G, double rs, int64_t nt,
            const int64_t *targets, double *acc, double *pot)
{
    int64_t n3 = (int64_t)ng * ng * ng;
    double *rho = (double *)malloc((size_t)n3 * sizeof(double));
    double *phi = (double *)malloc((size_t)n3 * sizeof(double));
    double *fx = (double *)malloc((size_t)n3 * sizeof(double));
    double *fy = (double *)malloc((size_t)n3 * sizeof(double));
    double *fz = (double *)malloc((size_t)n3 * sizeof(double));
    orc_cic_deposit(n, x, y, z, mass, box, ng, rho);
    orc_pm_mesh(ng, box, G, rs, rho, phi, fx, fy, fz);
    const double *c[3] = {x, y, z};
    const double *F[3] = {fx, fy, fz};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nt; k++) {
        int64_t p = targets[k];
        int i0[3];
        double w[3];
        for (int a = 0; a < 3; a++)
            cic_weights(c[a][p], box, ng, &i0[a], &w[a]);
        for (int a = 0; a < 3; a++)
            acc[a * nt + k] = cic_interp(F[a], ng, i0, w);
        if (pot)
            pot[k] = cic_interp(phi, ng, i0, w);
    }
    free(rho);
    free(phi);
    free(fx);
    free(fy);
    free(fz);
}

/* ------------------------------------------------------------------ */
/* Particle-mesh long-range force without periodicity (Sec. 3.3: an   */
/* isolated system takes a padded mesh with its own Green's function). */
/*                                                                     */
/* The ng-cell mesh spans the root cube [x0, x0 + L) plus two cells on */
/* each side: h = L / (ng - 4), mesh origin x0 - 2h.  It is embedded in */
/* a (2 ng)^3 zero-padded mesh, so the circular convolution equals the */
/* open one for every mesh point the difference stencil reads.  Green's */
/* function: the long-range part of the point-mass potential,          */
/*   G_l(r) = -G erf(r / 2 r_s) / r,  G_l(0) = -G / (sqrt(pi) r_s),     */
/* sampled at the signed mesh offsets, transformed, and divided by the  */
/* CIC deconvolution prod_a sinc^4(k_a h / 2) (as in the periodic case).*/
/* Masses (not densities) are deposited, so                            */
/*   Phi = IFFT(FFT(M) FFT(G_l) / deconv) / (2 ng)^3.                   */
/* deconv = 0 skips the deconvolution (a test hook).                   */
/* Mesh indices are taken modulo 2 ng (the padded transform is         */
/* circular): a particle on the lower face of the root cube may round   */
/* into cell 1, and its stencil then reads index -1, which the spare    */
/* cells keep free of wrapped images.                                   */
/* ------------------------------------------------------------------ */
static int64_t pad_index(int M, int i, int j, int k)
{
    i = ((i % M) + M) % M;
    j = ((j % M) + M) % M;
    k = ((k % M) + M) % M;
    return ((int64_t)i * M + j) * M + k;
}

static double isolated_kernel(double r, double G, double rs)
{
    if (r == 0.0)
        return -G / (sqrt(M_PI) * rs);
    return -G * erf(r * (0.5 / rs)) / r;
}

void orc_pm_isolated(int64_t n, const double *x, const double *y, const double *z,
                     const double *mass, const double *frame /* x0, y0, z0, L */, int ng,
                     double G, double asmth, int deconv, int64_t nt, const int64_t *targets,
                     double *acc, double *pot)
{
    const int M = 2 * ng;
    const int64_t M3 = (int64_t)M * M * M;
    const double h = frame[3] / (ng - 4);
    const double rs = asmth * h;
    const double lo[3] = {frame[0] - 2.0 * h, frame[1] - 2.0 * h, frame[2] - 2.0 * h};
    double *re = (double *)calloc((size_t)M3, sizeof(double));
    double *im = (double *)calloc((size_t)M3, sizeof(double));
    double *gre = (double *)calloc((size_t)M3, sizeof(double));
    double *gim = (double *)calloc((size_t)M3, sizeof(double));
    /* 1. CIC deposit of the masses */
    const double *c[3] = {x, y, z};
    for (int64_t p = 0; p < n; p++) {
        int i0[3];
        double w[3];
        for (int a = 0; a < 3; a++) {
            double f = (c[a][p] - lo[a]) / h;
            double fl = floor(f);
            w[a] = f - fl;
            i0[a] = (int)fl;
        }
        double m = mass ? mass[p] : 1.0 / (double)n;
        for (int s = 0; s < 8; s++) {
            double wt = 1.0;
            int t[3];
            for (int a = 0; a < 3; a++) {
                int up = (s >> (2 - a)) & 1;
                wt *= up ? w[a] : 1.0 - w[a];
                t[a] = i0[a] + up;
            }
            re[pad_index(M, t[0], t[1], t[2])] += m * wt;
        }
    }
    /* 2. Green's function at the signed offsets of the padded mesh */
    for (int i = 0; i < M; i++)
        for (int j = 0; j < M; j++)
            for (int k = 0; k < M; k++) {
#if ORC_MUTATION == 11
                int o[3] = {i, j, k};
#else
                int o[3] = {i < ng ? i : i - M, j < ng ? j : j - M, k < ng ? k : k - M};
#endif
                double r = h * sqrt((double)o[0] * o[0] + (double)o[1] * o[1] +
                                    (double)o[2] * o[2]);
                gre[((int64_t)i * M + j) * M + k] = isolated_kernel(r, G, rs);
            }
    /* 3. forward transforms, product, deconvolution */
    orc_fft3(M, re, im, -1);
    orc_fft3(M, gre, gim, -1);
    for (int i = 0; i < M; i++)
        for (int j = 0; j < M; j++)
            for (int k = 0; k < M; k++) {
                int64_t q = ((int64_t)i * M + j) * M + k;
                int nn[3] = {i < ng ? i : i - M, j < ng ? j : j - M, k < ng ? k : k - M};
                double dc = 1.0;
                if (deconv)
                    for (int a = 0; a < 3; a++) {
                        double sarg = M_PI * nn[a] / M; /* k_a h / 2 */
                        double sc = nn[a] == 0 ? 1.0 : sin(sarg) / sarg;
                        dc *= sc * sc * sc * sc;
                    }
                double ar = re[q], ai = im[q];
                re[q] = (ar * gre[q] - ai * gim[q]) / dc;
                im[q] = (ar * gim[q] + ai * gre[q]) / dc;
            }
    free(gre);
    free(gim);
    /* 4. inverse transform */
    orc_fft3(M, re, im, +1);
    for (int64_t q = 0; q < M3; q++)
        re[q] /= (double)M3;
    free(im);
    double *phi = re;
    /* 5. four-point difference at the mesh points and 6. CIC interpolation */
#pragma omp parallel for schedule(static)
    for (int64_t kk = 0; kk < nt; kk++) {
        int64_t p = targets[kk];
        int i0[3];
        double w[3];
        for (int a = 0; a < 3; a++) {
            double f = (c[a][p] - lo[a]) / h;
            double fl = floor(f);
            w[a] = f - fl;
            i0[a] = (int)fl;
        }
        double F[3] = {0.0, 0.0, 0.0}, P = 0.0;
        for (int s = 0; s < 8; s++) {
            double wt = 1.0;
            int t[3];
            for (int a = 0; a < 3; a++) {
                int up = (s >> (2 - a)) & 1;
                wt *= up ? w[a] : 1.0 - w[a];
                t[a] = i0[a] + up;
            }
            for (int a = 0; a < 3; a++) {
                double v[5];
                for (int st = -2; st <= 2; st++) {
                    int u[3] = {t[0], t[1], t[2]};
                    u[a] += st;
                    v[st + 2] = phi[pad_index(M, u[0], u[1], u[2])];
                }
                double grad = ((2.0 / 3.0) * (v[3] - v[1]) - (1.0 / 12.0) * (v[4] - v[0])) / h;
                F[a] += wt * -grad;
            }
            P += wt * phi[pad_index(M, t[0], t[1], t[2])];
        }
        for (int a = 0; a < 3; a++)
            acc[a * nt + kk] = F[a];
        if (pot)
            pot[kk] = P;
    }
    free(re);
}

/* ------------------------------------------------------------------ */
/* Ewald summation (Sec. 3.1): exact periodic force with a uniform     */
/* neutralising background, split at sigma into a real-space sum over  */
/* images and a Fourier sum; plus the softening correction of nearby   */
/* pairs.  Independent of the PM code above (direct sums over k).      */
/* ------------------------------------------------------------------ */
void orc_ewald(int64_t n, const double *x, const double *y, const double *z,
               const double *mass, double box, double G, double eps, double sigma,
               int64_t nt, const int64_t *targets, double *acc)
{
    double h = 2.8 * eps;
    double rmax = 12.0 * sigma;
    int nimg = (int)ceil(rmax / box);
    double kmax = 6.5 / sigma;
    int nk = (int)ceil(kmax * box / (2.0 * M_PI));
    double V = box * box * box;
    /* structure factor over half of k-space (k and -k contribute alike) */
    int64_t nvec = 0;
    int64_t cap = (int64_t)(2 * nk + 1) * (2 * nk + 1) * (nk + 1);
    double *kv = (double *)malloc((size_t)(4 * cap) * sizeof(double));
    for (int a = -nk; a <= nk; a++)
        for (int b = -nk; b <= nk; b++)
            for (int c = 0; c <= nk; c++) {
                if (c == 0 && (b < 0 || (b == 0 && a <= 0)))
                    continue;
                double k[3] = {2 * M_PI * a / box, 2 * M_PI * b / box, 2 * M_PI * c / box};
                double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                if (k2 > kmax * kmax)
                    continue;
                kv[4 * nvec + 0] = k[0];
                kv[4 * nvec + 1] = k[1];
                kv[4 * nvec + 2] = k[2];
                kv[4 * nvec + 3] = 2.0 * 4.0 * M_PI * G / (V * k2) * exp(-k2 * sigma * sigma);
                nvec++;
            }
    double *Sc = (double *)calloc((size_t)nvec, sizeof(double));
    double *Ss = (double *)calloc((size_t)nvec, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nvec; v++) {
        double sc = 0.0, ss = 0.0;
        for (int64_t j = 0; j < n; j++) {
            double m = mass ? mass[j] : 1.0 / (double)n;
            double ph = kv[4 * v] * x[j] + kv[4 * v + 1] * y[j] + kv[4 * v + 2] * z[j];
            sc += m * cos(ph);
            ss += m * sin(ph);
        }
        Sc[v] = sc;
        Ss[v] = ss;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = targets[t];
        double a[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; j++) {
            double m = mass ? mass[j] : 1.0 / (double)n;
            double base[3] = {x[j] - x[i], y[j] - y[i], z[j] - z[i]};
            for (int c = 0; c < 3; c++)
                base[c] -= box * nearbyint(base[c] / box);
            for (int ia = -nimg; ia <= nimg; ia++)
                for (int ib = -nimg; ib <= nimg; ib++)
                    for (int ic = -nimg; ic <= nimg; ic++) {
                        if (j == i && ia == 0 && ib == 0 && ic == 0)
                            continue;
                        double d[3] = {base[0] + ia * box, base[1] + ib * box, base[2] + ic * box};
                        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                        if (r > rmax)
                            continue;
                        double s = r / (2.0 * sigma);
                        double f = G * m / (r * r * r) *
                                   (erfc(s) + 2.0 * s / sqrt(M_PI) * exp(-s * s));
                        if (r < h) { /* spline minus Newtonian, exact correction */
                            double u = r / h, g;
                            if (u < 0.5)
                                g = 32.0 / 3.0 - 192.0 / 5.0 * u * u + 32.0 * u * u * u;
                            else
                                g = 64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u * u -
                                    32.0 / 3.0 * u * u * u - 1.0 / (15.0 * u * u * u);
                            f += G * m * (g / (h * h * h) - 1.0 / (r * r * r));
                        }
                        for (int c = 0; c < 3; c++)
                            a[c] += f * d[c];
                    }
        }
        for (int64_t v = 0; v < nvec; v++) {
            double ph = kv[4 * v] * x[i] + kv[4 * v + 1] * y[i] + kv[4 * v + 2] * z[i];
            double s = sin(ph) * Sc[v] - cos(ph) * Ss[v];
            for (int c = 0; c < 3; c++)
                a[c] -= kv[4 * v + 3] * kv[4 * v + c] * s;
        }
        for (int c = 0; c < 3; c++)
            acc[c * nt + t] = a[c];
    }
    free(kv);
    free(Sc);
    free(Ss);
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0)
        omp_set_num_threads(k);
#else
    (void)k;
#endif
}
