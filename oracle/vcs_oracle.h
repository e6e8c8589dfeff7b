/*
 * Reference emulator ("the oracle") for the batched Atari VCS hot path.
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.
 */
#ifndef VCS_ORACLE_H
#define VCS_ORACLE_H
#include <stdint.h>

enum {
    ORC_MAPPER_2K = 0, ORC_MAPPER_4K = 1, ORC_MAPPER_F8 = 2, ORC_MAPPER_F6 = 3, ORC_MAPPER_F4 = 4,
    ORC_MAPPER_F8SC = 5, ORC_MAPPER_F6SC = 6, ORC_MAPPER_F4SC = 7, ORC_MAPPER_E0 = 8, ORC_MAPPER_COUNT = 9
};

/* action code of the console RESET switch held (joystick idle); 0..17 are the joystick actions */
enum { ORC_ACTION_RESET = 18 };
#define ORC_SC_SEED 0x5343534352414D00ull /* "SCSCRAM\0": seed offset of the Superchip RAM stream */

typedef struct Orc Orc;

Orc *orc_new(void);
void orc_free(Orc *m);
int orc_power_on(Orc *m, const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0, int ystart);
int orc_step_instruction(Orc *m);
void orc_run_cycles(Orc *m, int64_t budget);
void orc_set_action(Orc *m, int action);
void orc_set_draw_frame(Orc *m, int64_t frame);
void orc_env_step(Orc *m, int action, int frame_skip, int64_t step_index, int store_frame);
void orc_get_regs(const Orc *m, int64_t *out);
void orc_get_objects(Orc *m, int64_t *out);
void orc_op_stats(const Orc *m, uint64_t *out);
void orc_set_relax(Orc *m, int on, double alpha, double T);
int64_t orc_relax_ndiv(const Orc *m);
uint64_t orc_relax_fails(const Orc *m);
void orc_relax_last_dev(const Orc *m, double *out);
void orc_dispatch_deviation(const Orc *m, const double *logits, double T, double *dev, double *spread,
                            double *w_star);
const uint8_t *orc_ram(const Orc *m);
const uint8_t *orc_frame(const Orc *m);
void orc_poke_ram(Orc *m, int cell, int v);
int orc_intim_at(const Orc *m, int64_t t);
int orc_timint_at(const Orc *m, int64_t t);
int orc_opcode_info(int opcode, int *op, int *mode, int *cycles, int *page_penalty);
void orc_alu(int op, int a, int v, int p_in, int *result, int *p_out);
int orc_action_swcha(int action);
int orc_action_inpt4(int action);
void orc_splitmix_ram(uint64_t seed, uint64_t env, uint64_t episode, uint8_t *out);
void orc_splitmix_sc_ram(uint64_t seed, uint64_t env, uint64_t episode, uint8_t *out);
void orc_set_sc_ram(Orc *m, const uint8_t *v);
const uint8_t *orc_sc_ram(const Orc *m);
uint64_t orc_splitmix_next(uint64_t *state);
double orc_gate(double z, double alpha);
double orc_gate_grad(double z, double alpha);

int orc_run_env(const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0, const uint8_t *actions,
                int steps, int frame_skip, int ystart, const uint32_t *ep_steps, int n_episodes, uint64_t seed,
                int64_t env_index, uint8_t *ram_out, uint8_t *frame_out, int frames_mode, uint8_t *done_out,
                int64_t *final_regs, uint64_t *instructions, uint8_t *step_state);

void orc_decode_logit_rows(const float *rows, int64_t n, int k, double tau, uint8_t *hard, double *ev, double *mx,
                           double *z);
void orc_decode_tape_rows(const float *rows, int64_t n, uint8_t *hard, double *ev);
void orc_decode_action_rows(const float *rows, int64_t n, double tau, uint8_t *hard, double *e_swcha,
                            double *e_inpt4);
void orc_epilogue_rom(const float *logits, int64_t n, double tau, const double *g, double *out);
void orc_epilogue_tape(int64_t n, const double *g0, double *out);
void orc_epilogue_action(const float *logits, int64_t n, double tau, const double *g_swcha, const double *g_inpt4,
                         double *out);
int orc_soft_env(const uint8_t *rom_hard, const double *rom_ev, int rom_size, int mapper, const uint8_t *ram0_hard,
                 const double *ram0_ev, const uint8_t *act_hard, const double *swcha_ev, const double *inpt4_ev,
                 int steps, int frame_skip, int ystart, int mode, const double *grad_frame, const double *grad_ram,
                 uint8_t *ram_out, uint8_t *frame_out, double *ram_smooth, double *frame_smooth, double *g_rom,
                 double *g_ram0, double *g_swcha, double *g_inpt4, int64_t *n_nodes);
int orc_soft_env_from(const uint8_t *rom_hard, const double *rom_ev, int rom_size, int mapper,
                      const uint8_t *ram0_hard, const double *ram0_ev, int pre_steps, const uint8_t *pre_actions,
                      const uint8_t *act_hard, const double *swcha_ev, const double *inpt4_ev, int steps,
                      int frame_skip, int ystart, int mode, double read_T, const double *grad_frame,
                      const double *grad_ram, uint8_t *ram_out, uint8_t *frame_out, double *ram_smooth,
                      double *frame_smooth, double *g_rom, double *g_ram0, double *g_swcha, double *g_inpt4,
                      double *g_pos, double *frame_dpos, int64_t *n_nodes);
#endif
