/*
 * orc.h -- FP64 CPU oracle of the Barnes-Hut step with index interaction
 * lists and list reuse (Iwasawa et al. 2019, "Accelerated FDPS").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path never includes, links or calls anything declared here, and this code
 * includes nothing from the GPU path.
 *
 * Conventions
 *   - Particle positions/masses are FP64, G is an explicit argument.
 *   - "input order" = the order of the arrays handed to orc_build.
 *   - "sorted order" = Morton order produced by the stable key sort; list
 *     ids for particles (EPJ) are sorted-order positions, list ids for
 *     superparticles (SPJ) are cell ids (cells numbered in DFS pre-order).
 *   - Every function returns 0 on success and a negative value on bad input
 *     (NULL pointer, negative size, allocation failure).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_tree orc_tree;

/* Key helpers (section 4.3, local tree step 1). */
int orc_root(int64_t n, const double* x, const double* y, const double* z,
             double lo[3], int* k);
int orc_keys(int64_t n, const double* x, const double* y, const double* z,
             const double lo[3], int k, uint64_t* key);
uint64_t orc_interleave(uint32_t qx, uint32_t qy, uint32_t qz);
void orc_deinterleave(uint64_t key, int level, uint32_t q[3]);

/* Tree: root cell, keys, sort, reorder, link, moments, groups
 * (section 4.3 local tree steps 1-4 and the moment pass). */
orc_tree* orc_build(int64_t n, const double* x, const double* y,
                    const double* z, const double* m, int n_leaf, int n_grp);
void orc_free(orc_tree* t);
/* info[0]=n info[1]=n_cell info[2]=n_groups info[3]=k info[4]=n_leaf
 * info[5]=n_grp; lo[3] = root corner. */
int orc_info(const orc_tree* t, int64_t info[6], double lo[3]);
int orc_get_keys(const orc_tree* t, uint64_t* key, uint32_t* perm);
int orc_get_cells(const orc_tree* t, uint64_t* prefix, uint8_t* level,
                  uint32_t* begin, uint32_t* count, uint32_t* parent,
                  uint32_t* skip, uint8_t* leaf, double* ctr3);
int orc_get_moments(const orc_tree* t, double* mass, double* com3,
                    double* quad6);
int orc_get_groups(const orc_tree* t, uint32_t* cell, uint32_t* begin,
                   uint32_t* count, double* lo3, double* hi3, double* ctr3);

/* Interaction lists (section 4.1 indirect addressing, section 4.3 list
 * construction).  sel == NULL walks every group; otherwise only the n_sel
 * listed groups, and the CSR is over that selection. */
int orc_make_lists(orc_tree* t, double theta, int64_t n_sel,
                   const int64_t* sel, int64_t sizes[3]);
int orc_get_lists(const orc_tree* t, int64_t* epj_off, uint32_t* epj,
                  int64_t* spj_off, uint32_t* spj);

/* Reuse with per-group list refresh (an extension of section 4.2's list
 * reuse).  Cells keep their particle ranges; in every opening test the
 * geometric centre of a cell is moved by the displacement of its centre of
 * mass since construction (zero right after construction), and the cell's
 * side is replaced by twice the largest per-axis distance from that centre
 * to the box of its current particles when that is larger (never right
 * after construction).  Positions come from the last orc_build /
 * orc_refresh.  All but orc_cell_sides need lists of every group. */

/* The side each cell has in the opening test now (n_cell values). */
int orc_cell_sides(const orc_tree* t, double* side);

/* Opening-test slacks of the walk that made each group's list: sa = the
 * smallest |box - centre| - rcrit over accepted cells, so = the smallest
 * rcrit - |box - centre| over opened cells that do not hold the group;
 * +inf when there is no such cell. */
int orc_group_margins(const orc_tree* t, double* sa, double* so);

/* stale[g] = 1 when a superparticle of the group's kept list fails the
 * opening test at angle theta (1 + tau), tau >= 0, measured from the
 * group's current tight box.  lo3/hi3 (current boxes) may be NULL. */
int orc_group_stale(const orc_tree* t, double theta, double tau,
                    uint8_t* stale, double* lo3, double* hi3);

/* Walk the n_sel listed groups (ascending ids) again with their current
 * boxes, keep every other list.  sizes = {n_groups, n_epj, n_spj}. */
int orc_refresh_lists(orc_tree* t, double theta, int64_t n_sel,
                      const int64_t* sel, int64_t sizes[3]);

/* The 12 predictor inputs per group (definitions in orc.c); age[g] = reuse
 * steps since the group's list was walked, kmax >= 1. */
int orc_group_features(const orc_tree* t, int kmax, const int32_t* age,
                       double* feat);

/* Rebuild predictor (mlp.c): 12-64-64-1 perceptron, tanh hidden layers,
 * logistic output, mean binary cross-entropy, Adam.  Parameter layout:
 * W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3.  pos_weight
 * multiplies the loss terms of positive labels. */
int orc_mlp_nparam(void);
int orc_mlp_forward(const double* w, int64_t n, const double* x, double* p);
int orc_mlp_loss_grad(const double* w, int64_t n, const double* x,
                      const double* y, double pos_weight, double* loss,
                      double* grad);
int orc_adam(double* w, const double* g, double* m, double* v, int64_t t,
             double lr, double beta1, double beta2, double eps);

/* Reuse step (section 4.2): new positions/masses in INPUT order; the tree
 * topology, cell geometry, groups and lists stay frozen, moments are
 * recomputed over the frozen particle ranges. */
int orc_refresh(orc_tree* t, const double* x, const double* y,
                const double* z, const double* m);

/* Forces from the saved lists of the selected groups (selection used by the
 * last orc_make_lists).  order 1 = monopole SPJ, 2 = quadrupole SPJ.
 * Outputs are written in INPUT order for members of the walked groups
 * only; other entries are left untouched. */
int orc_force_lists(const orc_tree* t, int order, double eps, double G,
                    double* ax, double* ay, double* az, double* pot);

/* Direct O(N^2) sum over all j != i for the n_tgt targets (input indices);
 * outputs are indexed like tgt (length n_tgt). */
int orc_force_direct(int64_t n, const double* x, const double* y,
                     const double* z, const double* m, double eps, double G,
                     int64_t n_tgt, const int64_t* tgt, double* ax,
                     double* ay, double* az, double* pot);

/* Kick-drift of the KDK leapfrog: v += a*dt_kick (plus the pull of a fixed
 * point mass ext_mass at the origin), then x += v*dt_drift. */
int orc_kick_drift(int64_t n, double* x, double* y, double* z, double* vx,
                   double* vy, double* vz, const double* ax,
                   const double* ay, const double* az, double dt_kick,
                   double dt_drift, double ext_mass, double G);

/* Threads the OpenMP runtime gives the per-group loops. */
int orc_num_threads(void);

/* Short-range interactions (section 2, section 4.2).  Neighbour lists for
 * search radius h over every group (EPJ only, sorted-order ids); the SPH
 * kernel W(r, h); densities over the lists (input order) and over all
 * pairs. */
int orc_neighbour_lists(orc_tree* t, double h, int64_t* n_entries);
int orc_get_neighbour_lists(const orc_tree* t, int64_t* off, uint32_t* ids);
double orc_sph_w(double r, double h);
int orc_sph_density(const orc_tree* t, double h, double* rho);
int orc_sph_density_direct(int64_t n, const double* x, const double* y,
                           const double* z, const double* m, double h,
                           double* rho);

#ifdef __cplusplus
}
#endif
#endif
