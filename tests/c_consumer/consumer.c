/* A C consumer of libqgbe: compiled against include/qgbe.h with a plain C
 * compiler and linked to the library, it prints the layout of every struct
 * the header declares and calls the two host-only helpers (no device needed).
 * tests/test_c_consumer.py compares the layouts with the ctypes binding and
 * the helpers' results with the oracle. */
#include <stddef.h>
#include <stdio.h>
#include "qgbe.h"

#define FIELD(T, f) printf("%s.%s %zu %zu\n", #T, #f, offsetof(T, f), sizeof(((T*)0)->f))

int main(void) {
  printf("sizeof qgbe_grid_desc %zu\n", sizeof(qgbe_grid_desc));
  FIELD(qgbe_grid_desc, n_x); FIELD(qgbe_grid_desc, n_p); FIELD(qgbe_grid_desc, x_half);
  FIELD(qgbe_grid_desc, p_half); FIELD(qgbe_grid_desc, species_mask); FIELD(qgbe_grid_desc, row_mask);
  FIELD(qgbe_grid_desc, alpha_s); FIELD(qgbe_grid_desc, precision); FIELD(qgbe_grid_desc, symmetric);
  FIELD(qgbe_grid_desc, drift); FIELD(qgbe_grid_desc, mass_mode); FIELD(qgbe_grid_desc, const_mass2);
  FIELD(qgbe_grid_desc, seed); FIELD(qgbe_grid_desc, device); FIELD(qgbe_grid_desc, stream);
  printf("sizeof qgbe_stats %zu\n", sizeof(qgbe_stats));
  FIELD(qgbe_stats, N_total); FIELD(qgbe_stats, N); FIELD(qgbe_stats, E_total); FIELD(qgbe_stats, E);
  FIELD(qgbe_stats, P); FIELD(qgbe_stats, mass2_avg); FIELD(qgbe_stats, min_f); FIELD(qgbe_stats, max_fermion_f);
  FIELD(qgbe_stats, n_evals); FIELD(qgbe_stats, t_collide_ms); FIELD(qgbe_stats, t_step_ms);
  FIELD(qgbe_stats, flags); FIELD(qgbe_stats, step); FIELD(qgbe_stats, n_accepted); FIELD(qgbe_stats, mc_err_est);
  FIELD(qgbe_stats, E_source); FIELD(qgbe_stats, E_collide); FIELD(qgbe_stats, E_total_mod);
  FIELD(qgbe_stats, entropy); FIELD(qgbe_stats, T_ii);
  FIELD(qgbe_stats, n_collide_launches); FIELD(qgbe_stats, reserved);
  printf("sizeof qgbe_collide_extras %zu\n", sizeof(qgbe_collide_extras));
  FIELD(qgbe_collide_extras, scale); FIELD(qgbe_collide_extras, item_sums); FIELD(qgbe_collide_extras, on_device);
  printf("sizeof qgbe_train_cfg %zu\n", sizeof(qgbe_train_cfg));
  FIELD(qgbe_train_cfg, epochs); FIELD(qgbe_train_cfg, batch); FIELD(qgbe_train_cfg, lr);
  FIELD(qgbe_train_cfg, lr_final); FIELD(qgbe_train_cfg, alpha); FIELD(qgbe_train_cfg, seed);
  printf("const QGBE_MLP_PARAMS %d\n", QGBE_MLP_PARAMS);
  printf("const QGBE_MLP_BATCH %d\n", QGBE_MLP_BATCH);

  /* host helpers */
  int32_t rows[128 * 5];
  double w[128 * 2];
  const int32_t n = qgbe_channel_table(0x7Fu, 0x7Fu, rows, w, 128);
  printf("channels %d\n", n);
  for (int i = 0; i < n; ++i)
    printf("chan %d %d %d %d %d %.17g %.17g\n", rows[5 * i], rows[5 * i + 1], rows[5 * i + 2], rows[5 * i + 3],
           rows[5 * i + 4], w[2 * i], w[2 * i + 1]);
  printf("too_small %d\n", qgbe_channel_table(0x7Fu, 0x7Fu, rows, w, 3));
  const uint32_t ctr[4] = {0x243f6a88u, 0x85a308d3u, 0x13198a2eu, 0x03707344u};
  const uint32_t key[2] = {0xa4093822u, 0x299f31d0u};
  uint32_t out[4];
  qgbe_philox4x32_10(ctr, key, out);
  printf("philox %u %u %u %u\n", out[0], out[1], out[2], out[3]);
  return 0;
}
