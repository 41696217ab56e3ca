/*
 * ludax.h -- C ABI of the MI355X batched board-game engine.
 *
 * The library runs the data-parallel hot path of Ludax (Todd et al.,
 * "Ludax: A GPU-Accelerated Description Language for Board Games",
 * arXiv 2506.22609) as hand-written HIP kernels for gfx950: the start
 * position, the legal-action mask, the transition (placement, Connect Four's
 * gravity placement, Reversi's flanking flips and forced pass), the ordered
 * end rules (n-in-a-row, exactly five, Hex edge-to-edge connection, disc
 * count) and the uniform-random playout loop built on them, for many
 * environments at once.
 *
 * Games and sizes (App. C rule texts):
 *   LUDAX_TICTACTOE    3x3, a line of three wins, full board draws
 *   LUDAX_CONNECT_FOUR 6x7, placement on the floor or on a piece (Sec. 3.4),
 *                      a line of four or more wins, full board draws
 *   LUDAX_HEX          NxN, 1 <= N <= 19, parallelogram of hexagons, player 1
 *                      joins the top and bottom rows, player 2 the left and
 *                      right columns; no draws, no swap rule
 *   LUDAX_REVERSI      8x8, standard four-disc start, placements must flank,
 *                      all flanked lines flip, forced pass, the game ends when
 *                      both players pass in a row, most discs wins
 *   LUDAX_GOMOKU       NxN, 5 <= N <= 19, a line of exactly five wins, full
 *                      board draws
 *   LUDAX_YAVALATH     DxD, D = 3, 5, 7 or 9: a regular hexagon of diameter D
 *                      (61 cells for D = 9), four in a row wins, else three
 *                      in a row loses, full board draws.  Cells are numbered
 *                      row by row from the top, row r holding
 *                      D - |r - (D-1)/2| cells, left to right; lines run
 *                      along the rows and the two other hexagon axes.
 *   LUDAX_PENTE        NxN, N = 7, 9 or 19: the first stone goes to the exact
 *                      centre (the only legal placement on an empty board);
 *                      a placement bracketing exactly two opponent stones
 *                      against one of the mover's stones on a straight line
 *                      removes them; five or more in a row, or 10 captured
 *                      stones, wins; full board draws.  The state's `passes`
 *                      byte holds the captured pairs (player 1: low four
 *                      bits, player 2: high four bits); natural ply bound
 *                      cells + 16.
 *   LUDAX_WOLF_SHEEP   8x8 movement game (Sec. 3.2 step mechanic): player 1's
 *                      four sheep (cell value 1) start on cells 56, 58, 60,
 *                      62 and step diagonally up into an empty cell; player
 *                      2's wolf (value 2) starts on cell 3 and steps to any
 *                      empty diagonal neighbour.  The wolf wins on reaching
 *                      the bottom row; a player left without a legal move
 *                      after the opponent's ply loses.  Natural ply bound 56.
 *   LUDAX_DRAUGHTS     8x8 English Draughts (App. A listing): pawns (1, 2)
 *                      step diagonally forward (player 1 up, player 2 down)
 *                      or hop over an adjacent opponent piece into the empty
 *                      cell beyond and capture it; kings (cell value owner |
 *                      4: 5, 6) do both in all four diagonal directions.
 *                      While any hop is legal no step is.  After a ply a pawn
 *                      on its far row becomes a king; then, after a hop, if
 *                      the same piece can hop again the mover plays again
 *                      with that piece only: `passes` holds its cell + 1 (0
 *                      otherwise) and to_move stays.  A player left without
 *                      a legal move loses.  Natural ply bound: 200 (the
 *                      game itself is unbounded).
 *   LUDAX_HASAMI_SHOGI 9x9 Dai Hasami Shogi (Sec. 3.2 slide and hop): player
 *                      1's 18 pieces start on rows 7-8, player 2's on rows
 *                      0-1.  A piece slides any number of empty cells along
 *                      its row or column, or hops over an adjacent piece of
 *                      either player (no capture) to the empty cell beyond.
 *                      Every row or column run of opponent pieces enclosed
 *                      between the moved piece and another of the mover's
 *                      is captured, as is an opponent corner piece whose two
 *                      neighbours become the mover's.  Five of the mover's
 *                      pieces in a row or column, none on its two start
 *                      rows, win; a player left without a legal move loses.
 *                      Natural ply bound: 200 (unbounded game).
 * Anything else is LUDAX_E_UNSUPPORTED.
 *
 * Board and action conventions:
 *   cell (r, c) has index r*cols + c, r = 0 the top row, c = 0 the left
 *   column (Yavalath: the hexagon numbering above); a cell holds 0 (empty),
 *   1 (player 1) or 2 (player 2).
 *   The action space is the set of cells (Sec. 3.4: its size depends only
 *   on the board and the play mechanic), plus one PASS action at index
 *   rows*cols for Reversi.  For the movement games it is the set of
 *   ordered cell pairs: action src * cells + dst moves the piece on src to
 *   dst (4096 actions on 8x8, 6561 on 9x9).  Player 1 moves first; movers alternate; a pass
 *   is a ply.  Reversi: player 1 is black; discs start on D5, E4 (player 1)
 *   and D4, E5 (player 2) with letters naming columns left to right and
 *   digits rows top to bottom.
 *
 * Memory and streams: every buffer is caller-owned DEVICE memory; the
 * library never allocates, frees or synchronises inside ludax_init,
 * ludax_legal_mask, ludax_step or ludax_playout.  Work is enqueued on the
 * given stream and runs asynchronously; results are valid once the stream
 * has reached that point.  A game handle is immutable after creation and
 * may be used from several streams and threads at once.
 *
 * Errors: every call returns LUDAX_OK or a negative code.  Argument errors
 * are found on the host before anything is enqueued.  n = 0 is a no-op that
 * succeeds whatever the buffer pointers are (the game handle must be
 * valid).  Per-environment conditions (an illegal action, stepping an ended
 * environment) are found on the device and reported as data in the state,
 * never as return codes.
 */
#ifndef LUDAX_H
#define LUDAX_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* game kinds */
#define LUDAX_TICTACTOE    1
#define LUDAX_CONNECT_FOUR 2
#define LUDAX_HEX          3
#define LUDAX_REVERSI      4
#define LUDAX_GOMOKU       5
#define LUDAX_YAVALATH     6
#define LUDAX_PENTE        7
#define LUDAX_WOLF_SHEEP   8
#define LUDAX_DRAUGHTS     9
#define LUDAX_HASAMI_SHOGI 10

/* per-environment status values (ludax_state.status) */
#define LUDAX_RUNNING   0 /* the game goes on */
#define LUDAX_TERMINAL  1 /* an end rule fired; winner is 0 (draw), 1 or 2 */
#define LUDAX_TRUNCATED 2 /* max_plies reached without an end rule; winner -1 */
#define LUDAX_ILLEGAL   3 /* an action outside the legal mask was applied */

/* return codes */
#define LUDAX_OK             0
#define LUDAX_E_INVALID     -1 /* NULL required pointer, n < 0, misaligned board, bad desc */
#define LUDAX_E_UNSUPPORTED -2 /* unknown kind or unsupported board size */
#define LUDAX_E_DEVICE      -3 /* a HIP launch failed; see ludax_last_device_error() */

typedef struct ludax_game ludax_game; /* opaque, immutable after create */

/* Static description of a game (Sec. 4: every shape is fixed when the
 * game is built). */
typedef struct {
    int32_t kind;      /* LUDAX_TICTACTOE ... LUDAX_HASAMI_SHOGI */
    int32_t rows;
    int32_t cols;
    int32_t max_plies; /* 0 = the natural bound: cells (Reversi 121, Pente cells + 16,
                          Wolf and Sheep 56, Draughts and Dai Hasami Shogi 200);
                          at most 32767 */
} ludax_game_desc;

/* Structure-of-arrays batch state for n environments (Sec. 4, dynamic
 * state attributes: only the fields these games need).  All pointers are
 * device memory owned by the caller.  board must be 16-byte aligned.
 * States are expected to be reachable from ludax_init by steps and
 * playouts; on hand-edited boards results are defined only as "no memory
 * access outside the buffers" (see ludax_playout for the one safeguard). */
typedef struct {
    int8_t  *board;       /* [n][rows*cols], 0 empty, 1, 2 (Draughts kings: 5, 6) */
    int8_t  *to_move;     /* [n] player to move, 1 or 2 */
    int8_t  *status;      /* [n] LUDAX_RUNNING ... LUDAX_ILLEGAL */
    int8_t  *winner;      /* [n] -1 none, 0 draw, 1, 2 */
    int8_t  *passes;      /* [n] the game's extra state byte: Reversi's consecutive passes,
                             Pente's captured pairs, Draughts' extra-turn piece + 1
                             (see above), 0 otherwise */
    int16_t *ply;         /* [n] plies applied since the start */
    int16_t *last_action; /* [n] last applied action, -1 before the first */
    void    *aux;         /* NULL, or [n][aux_bytes] device bytes (128-byte aligned) of a
                             library-private per-env cache; see "aux" below */
} ludax_state;

/* aux: Hex keeps its connected components from ply to ply (Sec. 4, dynamic
 * state attributes: the `connected` end rule is served by a component
 * array that each move updates locally).  For Hex, aux_bytes > 0 and a
 * non-NULL state.aux holds, per env, both players' stones as bitboards and
 * a union-find over the stones with the side flags of each component.
 * ludax_init writes it; ludax_step, ludax_random_step and ludax_policy_step
 * then read the stones from it instead of the board and decide the end
 * test by joining the new stone to its neighbours' components (the board
 * is still updated, results are identical to aux = NULL).  Every call that
 * changes the state must pass the same aux; after any other change (a call
 * with aux = NULL, ludax_playout, a copy of states from elsewhere) call
 * ludax_aux_sync, or pass aux = NULL.  As a safeguard the cache records the
 * (ply, last_action) it belongs to, and a step that finds them changed
 * rebuilds that env's cache from the board first.  Every other call and
 * game ignores aux (aux_bytes = 0). */

/* Build a game handle.  Host only, no device work.  *out is set on
 * success; release it with ludax_game_destroy. */
int ludax_game_create(const ludax_game_desc *desc, ludax_game **out);
int ludax_game_destroy(ludax_game *game);

/* Shapes of a game: cells = rows*cols, num_actions = A, aux_bytes per env
 * (Hex: the size of its component cache, a multiple of 128; 0 for the other
 * games), max_plies after resolving 0 to the natural bound.  Any output
 * pointer may be NULL. */
int ludax_game_info(const ludax_game *game, int32_t *cells, int32_t *num_actions,
                    int32_t *aux_bytes, int32_t *max_plies);

/* Start position (Sec. 3.1 start rules) for all n environments: empty
 * board (Reversi: the four start discs; the movement games: their start
 * pieces), to_move 1, RUNNING, winner -1, passes 0, ply 0, last_action -1;
 * and the start of state.aux when it is used (Hex). */
int ludax_init(const ludax_game *game, ludax_state *state, int64_t n, hipStream_t stream);

/* Legal-action mask (Sec. 3.2: each play mechanic defines one of fixed
 * size).  mask: [n][A] uint8, 1 = legal.  An environment that is not
 * RUNNING has an all-zero row; a RUNNING one always has at least one legal
 * action (Reversi: PASS is legal exactly when no placement is). */
int ludax_legal_mask(const ludax_game *game, const ludax_state *state, uint8_t *mask, int64_t n,
                     hipStream_t stream);

/* One transition per environment (Sec. 3.2 mechanic then effects, Sec. 3.3
 * end rules checked in order, wins before draws):
 *   - env not RUNNING: no change; reward 0/0; terminal 1.
 *   - action outside [0, A) or not legal: status = ILLEGAL, nothing else
 *     changes; reward 0/0; terminal 1.
 *   - else the action is applied, ply += 1, last_action = action, and the
 *     mover's end rules are checked.  A win gives reward +1 to the winner
 *     and -1 to the loser, a draw 0/0; to_move stays the mover.  Otherwise
 *     to_move passes to the other player and, if ply reaches max_plies,
 *     status = TRUNCATED (reward 0/0).
 * action: [n] int32; reward: [n][2] int8 (player 1, player 2); terminal:
 * [n] uint8 = (status != RUNNING) after the step; next_mask: [n][A] uint8
 * legal mask of the new state, or NULL. */
int ludax_step(const ludax_game *game, ludax_state *state, const int32_t *action, int8_t *reward,
               uint8_t *terminal, uint8_t *next_mask, int64_t n, hipStream_t stream);

/* Uniform-random playout of every RUNNING environment to its end (Sec. 6:
 * a uniformly random legal action each ply).  At each ply with legal mask
 * m and n_legal = popcount(m):
 *   w = word (ply mod 4) of Philox4x32-10(counter = (ply / 4, low and high
 *       32 bits of the game id, 0), key = (low and high 32 bits of seed)),
 *   k = (w * n_legal) >> 32 (64-bit product),
 *   action = the k-th (from 0) legal action in increasing index order,
 * then the ply is applied as in ludax_step.  The game id of env i is
 * game_id[i], or game_id_base + i if game_id is NULL; so a game's moves
 * depend only on (seed, game id, ply), not on its slot or the batch.
 * reward [n][2]: the rewards of the ply that ended the game inside this
 * call (0/0 for envs that were not RUNNING at the call).  terminal [n]: 1.
 * stats [4] int64 or NULL is ADDED to (the caller zeroes it):
 *   {plies applied, player-1 wins, player-2 wins, draws} over games that
 *   ended inside this call.  A RUNNING env with no legal action (only
 *   possible on a hand-edited board) is set ILLEGAL and stops. */
int ludax_playout(const ludax_game *game, ludax_state *state, uint64_t seed,
                  int64_t game_id_base, const int64_t *game_id, int8_t *reward,
                  uint8_t *terminal, int64_t *stats, int64_t n, hipStream_t stream);

/* Several batches played out by one kernel launch (Sec. 6 measures batches
 * of single games; a step of its benchmark plays several games' batches).
 * Kernels queued on one stream run one after the other, so batches
 * launched separately leave the chip to one batch's waves at a time (a
 * 65536-env batch has one wave per SIMD); in one grid the batches' waves
 * share the SIMDs.  Each batch's results are exactly those of, in order,
 * [ludax_init if from_start] and ludax_playout(game, state, seed,
 * game_id_base, NULL, reward, terminal, stats, n): from_start != 0 resets
 * every env to its game's start position inside the kernel, so no field of
 * the state is read.  The group kernel holds the fill-then-resolve games
 * Tic-Tac-Toe, Connect Four 6x7 and Hex 11x11; a call with any other game
 * runs the batches one after another (the same kernels as ludax_init and
 * ludax_playout).  The state's aux cache, if any, is left describing the
 * final boards (from_start) or as ludax_playout leaves it.
 * batches: 1 <= n_batches <= 4 host structs; batches must not share device
 * buffers; the batches' n add up to at most 2^31 - 1; a batch with n = 0
 * is skipped (its pointers are not checked). */
typedef struct {
    const ludax_game *game;
    ludax_state *state;
    int64_t n;
    int64_t game_id_base; /* game id of env i: game_id_base + i */
    int8_t *reward;       /* [n][2] as ludax_playout */
    uint8_t *terminal;    /* [n] */
    int64_t *stats;       /* [4] int64 added to as ludax_playout's, or NULL */
} ludax_batch;

int ludax_playout_batches(const ludax_batch *batches, int32_t n_batches, uint64_t seed, int32_t from_start,
                          hipStream_t stream);

/* One ply of the uniform-random policy of ludax_playout for every
 * environment (Sec. 6), with the state left in HBM between calls: a
 * RUNNING env draws the action of its current ply exactly as
 * ludax_playout does (same Philox word, same k-th legal action) and steps
 * as ludax_step does; a RUNNING env with no legal action is set ILLEGAL.
 * Repeating the call until no env is RUNNING gives the same states as one
 * ludax_playout with the same seed and game ids.  reward [n][2] and
 * terminal [n] as in ludax_step (an env that was not RUNNING: 0/0 and 1);
 * game ids as in ludax_playout. */
int ludax_random_step(const ludax_game *game, ludax_state *state, uint64_t seed,
                      int64_t game_id_base, const int64_t *game_id, int8_t *reward,
                      uint8_t *terminal, int64_t n, hipStream_t stream);

/* One ply drawn from a policy instead of uniformly (the move proposal of
 * a learned policy, Sec. 7): exactly ludax_random_step, except that a
 * RUNNING env with legal placements plays the first legal action a (in
 * increasing order) at which the running float32 sum of exp(logits[a] -
 * max) over the legal placements exceeds u * (their total), u = (w >> 8) /
 * 2^24 for the ply's Philox word w (the last legal placement if rounding
 * leaves none); with no legal placement (Reversi) it passes.  logits:
 * [n][A] float32 in action order (a PASS entry is ignored).  Movement
 * games: the same rule over their legal moves in increasing action order. */
int ludax_policy_step(const ludax_game *game, ludax_state *state, const float *logits, uint64_t seed,
                      int64_t game_id_base, const int64_t *game_id, int8_t *reward, uint8_t *terminal,
                      int64_t n, hipStream_t stream);

/* Counter reduction used by ludax_playout's stats, exposed on its own:
 * stats[0..3] += sign * (sum of ply, number of TERMINAL envs won by player
 * 1, won by player 2, drawn) over the n envs; sign is +1 or -1.  Calling
 * it with sign -1 before and +1 after any sequence of calls on the same
 * stream adds the plies applied and the games ended in between -- exactly
 * what ludax_playout's stats argument adds. */
int ludax_state_stats(const ludax_game *game, const ludax_state *state, int32_t sign, int64_t *stats,
                      int64_t n, hipStream_t stream);

/* Rebuild the aux cache of all n environments from their boards (Hex;
 * Sec. 4's component array recomputed from scratch, the lowest cell of each
 * component its root).  A no-op for games with aux_bytes = 0;
 * LUDAX_E_INVALID if the game has a cache and state.aux is NULL. */
int ludax_aux_sync(const ludax_game *game, ludax_state *state, int64_t n, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Mixed persistent batch.  Several rule sets share the device in one call:
 * the games of a batch are the ids id_base + j, j in [0, n_games), and game
 * id g has kind games[g mod n_kinds] and plays from that game's start
 * position under the uniform-random policy of ludax_playout (same Philox
 * convention, so game g's result equals a one-env ludax_playout with game
 * id g).  Each kind runs its own persistent kernel over `slots` lanes
 * (envs in flight); a lane whose game ends takes the kind's next game from
 * a queue (64 games per atomic), so no lane waits for the longest game of
 * a fixed batch.  The kinds' kernels run concurrently on internal streams
 * forked from and joined back into the caller's stream, so the whole call
 * can be captured into a graph and replayed.  They overlap only where each
 * internal stream has a hardware queue of its own: HIP spreads a process's
 * streams over GPU_MAX_HW_QUEUES queues (4 by default) and kernels sharing
 * a queue run one after the other, so a process with several mixed handles
 * or many other streams sets GPU_MAX_HW_QUEUES (up to 32) to at least its
 * number of streams before the runtime starts (1M-game 19x19 mixed batch:
 * 4.2 ms with both kinds' streams on one queue, 3.0 ms on two).
 * ------------------------------------------------------------------------ */
typedef struct ludax_mixed ludax_mixed;

/* 1 <= n_kinds <= 8 game handles (they must outlive the mixed handle).
 * Creates the internal streams and events; the default plan gives every
 * kind 65536 slots.  A mixed handle serves one host thread at a time. */
int ludax_mixed_create(const ludax_game *const *games, int32_t n_kinds, ludax_mixed **out);
int ludax_mixed_destroy(ludax_mixed *mixed);

/* Lanes per kind: multiples of 64, at least 64 and at most 2^24 each. */
int ludax_mixed_set_slots(ludax_mixed *mixed, const int32_t *slots);
int ludax_mixed_get_slots(const ludax_mixed *mixed, int32_t *slots);

/* How the kinds are launched.  one_grid = 1: every kind's persistent loop
 * in one grid (block ranges per kind, one launch on the caller's stream;
 * the kinds overlap whatever the hardware queues, as long as the grid is
 * resident at once: at most 4 waves per SIMD, i.e. 262144 slots in all on
 * 256 CUs).  Only for kinds in the one-grid kernel's list: Tic-Tac-Toe,
 * Connect Four 6x7, Reversi 8x8, Hex 11x11, Gomoku 15x15
 * (LUDAX_E_UNSUPPORTED otherwise).  one_grid = 0: one kernel per kind on
 * the internal streams.  The default is 1 where supported; the autotuner
 * times both and keeps the faster.  Results do not depend on it. */
int ludax_mixed_set_one_grid(ludax_mixed *mixed, int32_t one_grid);
int ludax_mixed_get_one_grid(const ludax_mixed *mixed, int32_t *one_grid);

/* Play every game of the batch to its end.  Device outputs indexed by j:
 * winner [n_games] int8 (0 draw, 1, 2; -1 if truncated at max_plies),
 * plies [n_games] int16 (plies of the game), last_action [n_games] int16.
 * stats [n_kinds][4] int64 or NULL is ADDED to per kind: {plies, player-1
 * wins, player-2 wins, draws}.  workspace: n_kinds uint32 device words
 * (queue counters, cleared by the call).  id_base >= 0 and
 * id_base + n_games < 2^62. */
int ludax_mixed_playout(ludax_mixed *mixed, uint64_t seed, int64_t id_base, int64_t n_games,
                        int8_t *winner, int16_t *plies, int16_t *last_action, int64_t *stats,
                        uint32_t *workspace, hipStream_t stream);

/* ludax_mixed_playout without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, serving loops,
 * harnesses that forbid hipMalloc).  The queue counters (one 32-bit word per
 * kind, at most 8 words = 32 bytes) live in a static device array of the
 * library, one copy per GPU, held until the process ends; the call looks up
 * its device address once per device and allocates nothing.  Every call on
 * one GPU shares those words: the call clears them (with a small kernel, no
 * memset) before its kernels use them, and calls that overlap in time on
 * one GPU (several streams or host threads) race and give wrong results.
 * Arguments and results as in ludax_mixed_playout; returns LUDAX_E_INVALID
 * for more kinds than scratch words (never, with the 8-kind limit). */
int ludax_mixed_playout_noalloc(ludax_mixed *mixed, uint64_t seed, int64_t id_base, int64_t n_games,
                                int8_t *winner, int16_t *plies, int16_t *last_action, int64_t *stats,
                                hipStream_t stream);

/* The slot autotuner: times each kind alone at total_slots / n_kinds lanes
 * (its work) and at half and twice that (how its time scales with its
 * lanes: T(S) ~ T(S0) (S / S0)^-beta, beta = 1 for a kind that turns every
 * lane into speed, near 0 for one bound by its longest games), then times
 * whole batches under candidate splits of total_slots: equal, proportional
 * to the work, to its square root, the proportional split with the
 * largest kind's share moved by +-25 %, and the occupancy plan that brings
 * every kind's fitted time to a common value with the lanes adding up to
 * total_slots (and that plan with the flattest-scaling kind's share moved
 * by +-25 %), each split launched as one grid (where supported) and as a
 * kernel per kind, each timed twice (the better run counts); then refines
 * the fastest split in its launch mode, moving each kind's share by -30 %
 * and +40 %, then by -15 % and +18 % (a move kept when the batch gets
 * faster); keeps the result as the handle's plan
 * (ludax_mixed_get_slots and ludax_mixed_get_one_grid read it).  Runs real
 * batches with the given
 * arguments (outputs are overwritten) and SYNCHRONISES the stream.
 * *best_ms (may be NULL) receives the chosen plan's time. */
int ludax_mixed_autotune(ludax_mixed *mixed, uint64_t seed, int64_t id_base, int64_t n_games,
                         int32_t total_slots, int8_t *winner, int16_t *plies, int16_t *last_action,
                         uint32_t *workspace, hipStream_t stream, float *best_ms);

/* ------------------------------------------------------------------------
 * Policy/value network (the learned part; the paper trains policy/value
 * agents on its environments in Sec. 7 with a ResNet, this is a small
 * convolutional one).  For an N x N board, N = 11 or 19:
 *   planes   3 planes in the mover's frame (the mover's stones, the
 *            opponent's, the empty cells); for player 2 the board is
 *            transposed and the colours exchanged (the Hex symmetry that
 *            maps player 2's left-right goal onto top-bottom);
 *   trunk    4 x (3x3 convolution, zero padding, 64 channels, ReLU);
 *   policy   one logit per cell (1x1 convolution);
 *   value    tanh(wv . (channel means) + bv), the expected outcome for the
 *            mover.
 * Conv weights and activations are bfloat16 (round to nearest even), every
 * sum float32, the heads float32.
 * params: float32 [n_params], in this order: W1 [64][3][3][3] (out, in,
 * row, column), b1 [64], W2..W4 [64][64][3][3] each followed by its bias
 * [64], wp [64], bp [1], wv [64], bv [1].
 * packed: a device buffer of packed_bytes holding the bfloat16 copies the
 * kernels read; ludax_net_pack (or ludax_net_adam) rewrites it from params.
 * workspace: a device buffer of at least ludax_net_workspace_bytes(n,
 * training) bytes, 256-byte aligned; its contents need not persist between
 * calls.  Calls on one stream may share it; calls that overlap on several
 * streams need one each.
 * ------------------------------------------------------------------------ */
typedef struct ludax_net ludax_net;

int ludax_net_create(int32_t rows, int32_t cols, ludax_net **out);
int ludax_net_destroy(ludax_net *net);
int ludax_net_info(const ludax_net *net, int64_t *n_params, int64_t *packed_bytes);
int ludax_net_workspace_bytes(const ludax_net *net, int64_t n, int32_t training, int64_t *bytes);
/* HBM-budget admission: *n = the largest batch whose workspace (training or
 * inference) fits in budget_bytes (0 if none).  Large-board batches that do
 * not fit are evaluated in chunks of this size. */
int ludax_net_max_batch(const ludax_net *net, int64_t budget_bytes, int32_t training, int64_t *n);
int ludax_net_pack(const ludax_net *net, const float *params, void *packed, hipStream_t stream);

/* Forward pass of n positions (board [n][N*N] int8 and to_move [n] int8, as
 * in ludax_state; to_move must be 1 or 2).  logits [n][N*N] float32 in
 * ACTION order (the cells of the board, not of the mover's frame); value
 * [n] float32, for the mover. */
int ludax_net_forward(const ludax_net *net, const float *params, const void *packed, const int8_t *board,
                      const int8_t *to_move, int64_t n, float *logits, float *value, void *workspace,
                      hipStream_t stream);

/* Loss and gradient of a batch of n samples (position, action[i] = the cell
 * played in it, which must be empty, z[i] = the final outcome for the mover,
 * +1 / 0 / -1):
 *   L = (1/n) sum_i (v_i - z_i)^2 + beta max(z_i - v_i, 0) (-log pi_i[action_i])
 * where pi_i is the softmax of the logits over the empty cells and the
 * weight max(z_i - v_i, 0) of the second term is held constant.  loss [2] float32
 * receives the two parts; grads [n_params] float32 is overwritten with dL /
 * d(params).  Gradients of the trunk flow through bfloat16: each layer's
 * pre-activation gradient is rounded to bfloat16 before it multiplies
 * anything.  n >= 1. */
int ludax_net_loss_grad(const ludax_net *net, const float *params, const void *packed, const int8_t *board,
                        const int8_t *to_move, const int16_t *action, const float *z, int64_t n, float beta,
                        float *loss, float *grads, void *workspace, hipStream_t stream);

/* One Adam step (Kingma & Ba, bias-corrected, step >= 1) on params with the
 * moments m, v [n_params] float32; then repacks into packed (if not NULL). */
int ludax_net_adam(const ludax_net *net, float *params, const float *grads, float *m, float *v, int32_t step,
                   float lr, float beta1, float beta2, float eps, void *packed, hipStream_t stream);

/* Value cutoff: an estimate of each env's final outcome for player 1.  A
 * TERMINAL env gives its result (+1 player 1 won, -1 player 2 won, 0 draw),
 * a RUNNING one the network's value mapped to player 1 (v if player 1 is
 * to move, else -v), any other status 0.  The board must be game's size
 * (rows = cols = N of the net). */
int ludax_net_estimate(const ludax_net *net, const float *params, const void *packed, const ludax_state *state,
                       int64_t n, float *estimate, void *workspace, hipStream_t stream);

/* One network-guided ply of every env (the move proposal of Sec. 7's
 * learned policy, fused into the step): the forward pass of this net on the
 * env's board, then exactly ludax_policy_step with those logits -- the same
 * Philox word, the same running-sum draw over the legal placements in
 * increasing action order, the same rules and outputs -- but the logits
 * never leave the chip: the kernel of the last layer and the heads writes
 * them to LDS and one lane per env draws and plays the ply there.  Results
 * are identical to ludax_net_forward followed by ludax_policy_step.
 * Supported: the 11x11 net with Hex 11x11 or Gomoku 11x11 (else
 * LUDAX_E_UNSUPPORTED).  reward [n][2], terminal [n] as in ludax_step; game
 * ids as in ludax_playout; workspace as for ludax_net_forward (inference
 * size of n).  A state with an aux cache is stepped without it (the cache's
 * tag check rebuilds it in a later step). */
int ludax_net_guided_step(const ludax_net *net, const float *params, const void *packed, const ludax_game *game,
                          ludax_state *state, uint64_t seed, int64_t game_id_base, const int64_t *game_id,
                          int8_t *reward, uint8_t *terminal, int64_t n, void *workspace, hipStream_t stream);

/* Network-guided playouts with a value cutoff, in one kernel (Sec. 7's
 * learned policy as the move proposal and its value as the cutoff):
 * `plies` times ludax_net_guided_step for every env (an env stops when its
 * game ends), then ludax_net_estimate of the resulting states, with the
 * same results bit for bit -- the states, and estimate [n] float32 (the
 * outcome for player 1 of an ended game, the network's value mapped to
 * player 1 for a running one, 0 for any other status).  A block keeps its
 * four boards and their activations on chip for all plies; the logits never
 * leave it and no workspace is needed.  Supported: the 11x11 net with Hex
 * or Gomoku 11x11 (else LUDAX_E_UNSUPPORTED); plies >= 0. */
int ludax_net_guided_playout(const ludax_net *net, const float *params, const void *packed, const ludax_game *game,
                             ludax_state *state, int32_t plies, uint64_t seed, int64_t game_id_base,
                             const int64_t *game_id, float *estimate, int64_t n, hipStream_t stream);

/* Text of a return code; never NULL. */
const char *ludax_strerror(int code);

/* Text of the last HIP error seen by a call on this thread ("" if none). */
const char *ludax_last_device_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LUDAX_H */
