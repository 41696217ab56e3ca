/*
 * ludax_ref.h -- plain CPU oracle of the batched board-game step and the
 * uniform-random playout (Ludax, arXiv 2506.22609).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct definition
 * that the GPU library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the GPU library, and the GPU library
 * never calls it.
 *
 * Conventions (the paper leaves them open; the reading taken is stated once
 * here and applied everywhere):
 *   - cell (r, c) has index r*W + c; r = 0 is the top row, c = 0 the left
 *     column.  Cell values: 0 empty, 1 player 1, 2 player 2.
 *   - the action space is the set of cells (Sec. 3.4), plus one PASS action
 *     at index H*W for Reversi (the force_pass mechanic, App. B grammar).
 *   - player 1 moves first; movers alternate strictly; a pass is a ply.
 *   - end rules are evaluated in order, wins before draws (Sec. 3.3).
 *   - random play draws one Philox4x32-10 word per ply (see ludax_ref_playout).
 *   - Yavalath (App. C) is played on a regular hexagon whose diameter D
 *     (rows = cols = D, odd) runs left to right: side S = (D + 1) / 2, rows
 *     r = 0..D-1 from the top, row r holding D - |r - (S-1)| cells, numbered
 *     row by row, left to right (61 cells for D = 9).  In axial coordinates
 *     cell i of row r has q = i + max(0, S-1-r); (r, q) touches (r, q+-1),
 *     (r-1, q), (r-1, q+1), (r+1, q-1), (r+1, q), and straight lines run
 *     along (0, 1), (1, 0) and (1, -1).
 *   - Pente (App. C), N x N with N odd: while the board is empty the only
 *     legal placement is the centre; a placement that brackets exactly two
 *     opponent stones between itself and one of the mover's stones on a
 *     straight line (any of 8 directions) removes them; five or more in a
 *     row, or 10 captured stones, wins; a full board draws.  The state's
 *     `passes` byte holds the captured PAIRS: player 1's in the low four
 *     bits, player 2's in the high four bits.  Natural ply bound: cells + 16
 *     (at most 16 stones are removed before somebody reaches 10).
 *   - Movement games (Sec. 3.2 move mechanic: step and hop), both 8 x 8
 *     with the dark squares at (r + c) odd:
 *     the action space is every ordered pair of cells, action
 *     src * cells + dst (4096 actions), a move of the piece on src to dst.
 *     A piece may step to an empty diagonal neighbour, or (Draughts) hop
 *     over a diagonally adjacent opponent piece to the empty cell beyond,
 *     removing it.  Pawns (and sheep) go forward only: up (towards row 0)
 *     for player 1, down for player 2; kings (and the wolf) go any diagonal
 *     way.  Hops have priority: while any hop is legal, no step is.
 *     After a ply the mover wins if the player to move next has no legal
 *     action (Draughts' end rule; the sheep's win by blocking the wolf).
 *   - Wolf and Sheep (App. C): player 1's four sheep (cell value 1) start
 *     on 56, 58, 60, 62, player 2's wolf (value 2) on 3; the wolf wins on
 *     reaching the bottom row (checked before the blocking rule).  A sheep
 *     moves at most 7 times, so a game has at most 56 plies.
 *   - English Draughts (App. A listing, App. C): cell value = owner | 4 for
 *     a king (1, 2 pawns; 5, 6 kings); pawns start on the cells the listing
 *     gives.  After a ply, a pawn on the far row becomes a king; then, if
 *     the ply was a hop and the same piece can hop again, the mover takes an
 *     extra turn in which only that piece moves: `passes` holds its cell + 1
 *     (0 when no extra turn is pending) and to_move does not change.  The
 *     game has no natural end, so plies are capped at 200 (the paper's cap
 *     for unbounded games, Sec. 6).
 *   - Dai Hasami Shogi (App. C), 9 x 9, action src * 81 + dst: player 1's
 *     18 pieces start on rows 7-8, player 2's on rows 0-1.  A piece slides
 *     any number of empty cells along its row or column, or hops over one
 *     adjacent piece of either player (no capture) to the empty cell beyond.
 *     After the move, every straight row or column run of opponent pieces
 *     enclosed between the moved piece and another of the mover's pieces is
 *     captured, and so is an opponent piece on a corner whose two neighbours
 *     are then both the mover's (the moved piece being one of them).  Five
 *     of the mover's pieces in a row or column, none on the mover's start
 *     rows, win; then a next player without a legal move loses.  No natural
 *     end: 200 plies.
 */
#ifndef LUDAX_REF_H
#define LUDAX_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* game kinds (App. C rule texts) */
#define LUDAX_REF_TICTACTOE    1
#define LUDAX_REF_CONNECT_FOUR 2
#define LUDAX_REF_HEX          3
#define LUDAX_REF_REVERSI      4
#define LUDAX_REF_GOMOKU       5
#define LUDAX_REF_YAVALATH     6
#define LUDAX_REF_PENTE        7
#define LUDAX_REF_WOLF_SHEEP   8
#define LUDAX_REF_DRAUGHTS     9
#define LUDAX_REF_HASAMI_SHOGI 10

/* env status */
#define LUDAX_REF_RUNNING   0
#define LUDAX_REF_TERMINAL  1
#define LUDAX_REF_TRUNCATED 2
#define LUDAX_REF_ILLEGAL   3

/* return codes */
#define LUDAX_REF_OK           0
#define LUDAX_REF_E_INVALID   -1
#define LUDAX_REF_E_UNSUPPORTED -2

typedef struct {
    int32_t kind;       /* one of LUDAX_REF_* kinds */
    int32_t rows;
    int32_t cols;
    int32_t max_plies;  /* 0 = the game's natural bound */
} ludax_ref_desc;

/* Structure-of-arrays batch state, n environments, host memory. */
typedef struct {
    int8_t  *board;        /* [n][rows*cols] */
    int8_t  *to_move;      /* [n] 1 or 2 */
    int8_t  *status;       /* [n] RUNNING/TERMINAL/TRUNCATED/ILLEGAL */
    int8_t  *winner;       /* [n] -1 none, 0 draw, 1, 2 */
    int8_t  *passes;       /* [n] per game: Reversi's consecutive passes,
                              Pente's captured pairs, Draughts' extra-turn
                              piece + 1 */
    int16_t *ply;          /* [n] plies applied so far */
    int16_t *last_action;  /* [n] -1 before the first ply */
} ludax_ref_state;

/* Validates a description and reports its shapes. */
int ludax_ref_info(const ludax_ref_desc *d, int32_t *cells, int32_t *num_actions,
                   int32_t *max_plies);

/* Start position (Sec. 3.1 start rules; Reversi's four stones, App. C). */
int ludax_ref_init(const ludax_ref_desc *d, ludax_ref_state *s, int64_t n);

/* Fixed-size legal-action mask [n][A] of 0/1 bytes (Sec. 3.2). */
int ludax_ref_legal_mask(const ludax_ref_desc *d, const ludax_ref_state *s,
                         uint8_t *mask, int64_t n);

/* One transition per env (Sec. 3.2 play mechanic, then effects, then the
 * ordered end rules of Sec. 3.3).  reward [n][2] int8, terminal [n],
 * next_mask [n][A] or NULL. */
int ludax_ref_step(const ludax_ref_desc *d, ludax_ref_state *s, const int32_t *action,
                   int8_t *reward, uint8_t *terminal, uint8_t *next_mask, int64_t n);

/* Uniform-random playout of every env to the end (Sec. 6 benchmark policy).
 * game_id may be NULL (then game_id_base + i).  stats [4] int64 or NULL is
 * ADDED to: {plies applied, P1 wins, P2 wins, draws}.  threads <= 1 runs
 * serially; otherwise contiguous env ranges run on that many pthreads. */
int ludax_ref_playout(const ludax_ref_desc *d, ludax_ref_state *s, uint64_t seed,
                      int64_t game_id_base, const int64_t *game_id, int8_t *reward,
                      uint8_t *terminal, int64_t *stats, int64_t n, int threads);

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void ludax_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The Philox word a playout draws for (seed, game_id, ply). */
uint32_t ludax_ref_draw(uint64_t seed, int64_t game_id, int32_t ply);

/* Enumeration helpers over the oracle's own step (single env at index 0 of s).
 * perft: number of action sequences of exactly `depth` plies that stay legal
 * and never pass through an ended game before the last ply.
 * count_games: every complete game from the state; by_len_winner is
 * [(max_len+1)][3] int64 indexed [len][winner] with winner 0 draw, 1, 2;
 * games that end truncated (or longer than max_len) are not tabulated and
 * their number is returned through *truncated.  Returns the number of
 * games. */
int64_t ludax_ref_perft(const ludax_ref_desc *d, const ludax_ref_state *s, int depth);
/* The same count over TURNS: the plies of an extra turn (Draughts) belong
 * to the turn they continue, so a multi-hop capture is one turn. */
int64_t ludax_ref_perft_turns(const ludax_ref_desc *d, const ludax_ref_state *s, int depth);
int64_t ludax_ref_count_games(const ludax_ref_desc *d, const ludax_ref_state *s,
                              int64_t *by_len_winner, int max_len, int64_t *truncated);

/* The game's win predicate for `who` on a bare board (lines for
 * Tic-Tac-Toe, Connect Four and Gomoku, connection for Hex); -1 for games
 * without one (Reversi) or bad arguments. */
int ludax_ref_holds_win(const ludax_ref_desc *d, const int8_t *board, int who);

/* Internal-consistency checks run inside step when enabled (e.g. the
 * opponent of the mover is never found lined up or connected). */
void ludax_ref_set_checks(int on);
int64_t ludax_ref_check_failures(void);

#ifdef __cplusplus
}
#endif
#endif
