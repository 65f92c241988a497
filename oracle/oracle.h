/* Butterfly-counting oracle: test infrastructure only (see oracle.c). */
#ifndef PB_ORACLE_H
#define PB_ORACLE_H
#include <stdint.h>

enum {
    ORC_SIDE_AUTO = 0,
    ORC_SIDE_U = 1,
    ORC_SIDE_V = 2,
    ORC_DEGREE = 3,
    ORC_APPROX_DEGREE = 4,
    ORC_CODEG = 5,
    ORC_APPROX_CODEG = 6
};

int orc_bf4(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
            int64_t *glob, int64_t *vert, int64_t *edge);
int orc_pairs(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
              int64_t *glob, int64_t *vert, int64_t *edge);
int orc_count(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
              int64_t *glob, int64_t *vert, int64_t *edge);
int orc_count_sample(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                     int64_t t_stride, int64_t *glob);
int orc_vside(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
              int64_t *v_off, uint32_t *v_adj);
int orc_vertex_one(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                   const int64_t *v_off, const uint32_t *v_adj, int64_t x, int64_t *out);
int orc_edge_one(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
                 const int64_t *v_off, const uint32_t *v_adj, int64_t e, int64_t *out);
int orc_wedges(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj,
               const uint32_t *rank, int64_t *total, int64_t *per_source);
int orc_rank(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj, int kind,
             uint32_t *rank);
uint64_t orc_splitmix(uint64_t seed, uint64_t i);
int orc_sparsify(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj, int kind, double p,
                 uint64_t seed, int64_t *out_off, uint32_t *out_adj, int64_t *kept);
int orc_tip(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj, int side, int64_t *tip,
            int64_t *rounds_out);
int orc_wing(int64_t n_u, int64_t n_v, const int64_t *u_off, const uint32_t *u_adj, int64_t *wing,
             int64_t *rounds_out);
#endif
