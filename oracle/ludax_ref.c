/*
 * ludax_ref.c -- plain CPU oracle of the batched board-game step and the
 * uniform-random playout (Ludax, arXiv 2506.22609).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the GPU library.  It is deliberately
 * slow: one env at a time, scalar loops over cells, full-board scans for
 * every end rule.  No bitboards, no precomputed tables.
 *
 * What each part follows:
 *   init          Sec. 3.1 (start rules); Reversi start squares, App. C.
 *   legal         Sec. 3.2 (play mechanic defines a fixed-size legal mask);
 *                 Sec. 3.4 (Connect Four as cell placement above a piece or
 *                 the floor); App. C rule texts; force_pass in the App. B
 *                 grammar.
 *   step          Sec. 3.2 (mechanic, then effects such as Reversi's flip),
 *                 Sec. 3.3 (end rules checked in order, wins before draws).
 *   win rules     App. C: lines of 3 / 4 in Tic-Tac-Toe / Connect Four,
 *                 exactly five in Gomoku, Hex edge-to-edge connection,
 *                 Reversi disc count after both players pass, Yavalath's
 *                 four in a row wins / three in a row (without four) loses,
 *                 Pente's five in a row or ten captured stones.
 *   movement      Sec. 3.2 (move mechanic: step, hop; hop priority over
 *                 step; capture, promotion and extra-turn effects), the App. A
 *                 English Draughts listing (start cells, effect order, end
 *                 rule) and the App. C rule texts of Wolf and Sheep and
 *                 English Draughts.
 *   playout       Sec. 6 (uniform-random action policy, full games).
 *   Philox        Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
 *                 Easy as 1, 2, 3", SC'11: Philox4x32 with 10 rounds.
 */
#include "ludax_ref.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define MAX_CELLS 361
#define MAX_ACTIONS 6561 /* 81 x 81 ordered cell pairs of Dai Hasami Shogi */

typedef struct {
    int kind, H, W, cells, A, max_plies;
    int S; /* Yavalath: side of the hexagon */
} game_t;

typedef struct {
    int8_t board[MAX_CELLS];
    int to_move, status, winner, passes, ply, last_action;
} env_t;

static volatile int g_checks = 0;
static int64_t g_check_failures = 0;
static pthread_mutex_t g_check_mu = PTHREAD_MUTEX_INITIALIZER;

void ludax_ref_set_checks(int on) { g_checks = on; }
int64_t ludax_ref_check_failures(void) { return g_check_failures; }

static void check_failed(void)
{
    pthread_mutex_lock(&g_check_mu);
    g_check_failures++;
    pthread_mutex_unlock(&g_check_mu);
}

/* ------------------------------------------------------------------ */
/* game descriptions                                                   */
/* ------------------------------------------------------------------ */

static int natural_bound(int kind, int cells)
{
    switch (kind) {
    case LUDAX_REF_REVERSI:
        /* 60 placements, at most 59 single passes between them, and the
         * final two passes. */
        return (cells - 4) + (cells - 4 - 1) + 2;
    case LUDAX_REF_PENTE:
        /* a capture frees two cells; after 16 removed stones somebody has
         * captured 10 and won, so the board fills by then */
        return cells + 16;
    case LUDAX_REF_WOLF_SHEEP:
        /* every other ply moves a sheep one row up, at most 7 rows each */
        return 2 * 4 * 7;
    case LUDAX_REF_DRAUGHTS:
    case LUDAX_REF_HASAMI_SHOGI:
        /* pieces can move back and forth forever: the paper's 200-turn cap */
        return 200;
    default:
        return cells; /* one stone per ply, never removed */
    }
}

static int resolve(const ludax_ref_desc *d, game_t *g)
{
    if (!d) return LUDAX_REF_E_INVALID;
    int k = d->kind, H = d->rows, W = d->cols;
    if (H <= 0 || W <= 0 || d->max_plies < 0 || d->max_plies > 32767) return LUDAX_REF_E_INVALID;
    int ok = 0;
    switch (k) {
    case LUDAX_REF_TICTACTOE:    ok = (H == 3 && W == 3); break;
    case LUDAX_REF_CONNECT_FOUR: ok = (H == 6 && W == 7); break;
    case LUDAX_REF_HEX:          ok = (H == W && H >= 1 && H <= 19); break;
    case LUDAX_REF_REVERSI:      ok = (H == 8 && W == 8); break;
    case LUDAX_REF_GOMOKU:       ok = (H == W && H >= 5 && H <= 19); break;
    case LUDAX_REF_YAVALATH:     ok = (H == W && (H & 1) && H >= 3 && H <= 9); break;
    case LUDAX_REF_PENTE:        ok = (H == W && (H & 1) && H >= 5 && H <= 19); break;
    case LUDAX_REF_WOLF_SHEEP:
    case LUDAX_REF_DRAUGHTS:     ok = (H == 8 && W == 8); break;
    case LUDAX_REF_HASAMI_SHOGI: ok = (H == 9 && W == 9); break;
    default: return LUDAX_REF_E_UNSUPPORTED;
    }
    if (!ok) return LUDAX_REF_E_UNSUPPORTED;
    g->kind = k;
    g->H = H;
    g->W = W;
    g->cells = H * W;
    g->S = 0;
    if (k == LUDAX_REF_YAVALATH) {
        g->S = (H + 1) / 2;
        g->cells = 3 * g->S * (g->S - 1) + 1;
    }
    g->A = g->cells + (k == LUDAX_REF_REVERSI ? 1 : 0);
    if (k == LUDAX_REF_WOLF_SHEEP || k == LUDAX_REF_DRAUGHTS || k == LUDAX_REF_HASAMI_SHOGI)
        g->A = g->cells * g->cells;
    g->max_plies = d->max_plies ? d->max_plies : natural_bound(k, g->cells);
    return LUDAX_REF_OK;
}

int ludax_ref_info(const ludax_ref_desc *d, int32_t *cells, int32_t *num_actions,
                   int32_t *max_plies)
{
    game_t g;
    int rc = resolve(d, &g);
    if (rc) return rc;
    if (cells) *cells = g.cells;
    if (num_actions) *num_actions = g.A;
    if (max_plies) *max_plies = g.max_plies;
    return LUDAX_REF_OK;
}

/* ------------------------------------------------------------------ */
/* state access                                                        */
/* ------------------------------------------------------------------ */

static int state_ok(const ludax_ref_state *s)
{
    return s && s->board && s->to_move && s->status && s->winner && s->passes && s->ply &&
           s->last_action;
}

static void load_env(const game_t *g, const ludax_ref_state *s, int64_t i, env_t *e)
{
    memcpy(e->board, s->board + i * g->cells, (size_t)g->cells);
    e->to_move = s->to_move[i];
    e->status = s->status[i];
    e->winner = s->winner[i];
    e->passes = s->passes[i];
    e->ply = s->ply[i];
    e->last_action = s->last_action[i];
}

static void store_env(const game_t *g, ludax_ref_state *s, int64_t i, const env_t *e)
{
    memcpy(s->board + i * g->cells, e->board, (size_t)g->cells);
    s->to_move[i] = (int8_t)e->to_move;
    s->status[i] = (int8_t)e->status;
    s->winner[i] = (int8_t)e->winner;
    s->passes[i] = (int8_t)e->passes;
    s->ply[i] = (int16_t)e->ply;
    s->last_action[i] = (int16_t)e->last_action;
}

static int on_board(const game_t *g, int r, int c) { return r >= 0 && r < g->H && c >= 0 && c < g->W; }

static int at(const game_t *g, const env_t *e, int r, int c) { return e->board[r * g->W + c]; }

/* ------------------------------------------------------------------ */
/* init                                                                */
/* ------------------------------------------------------------------ */

static void init_env(const game_t *g, env_t *e)
{
    memset(e->board, 0, sizeof e->board);
    if (g->kind == LUDAX_REF_REVERSI) {
        /* App. C: white on D4 and E5, black on D5 and E4.  Letters name
         * columns left to right, digits name rows top to bottom.  Player 1
         * is black and moves first. */
        const int D = 3, E = 4, row4 = 3, row5 = 4;
        e->board[row4 * 8 + D] = 2; /* D4 white */
        e->board[row5 * 8 + E] = 2; /* E5 white */
        e->board[row5 * 8 + D] = 1; /* D5 black */
        e->board[row4 * 8 + E] = 1; /* E4 black */
    }
    if (g->kind == LUDAX_REF_WOLF_SHEEP) {
        /* App. C: the sheep on the dark cells of the bottom row, the wolf on
         * a central dark cell of the top row (the left one of the two) */
        for (int c = 0; c < 8; c += 2) e->board[7 * 8 + c] = 1;
        e->board[3] = 2;
    }
    if (g->kind == LUDAX_REF_DRAUGHTS) {
        /* the start cells of the App. A listing: the dark cells of rows 5-7
         * for player 1 and of rows 0-2 for player 2 */
        static const int P1[12] = {40, 42, 44, 46, 49, 51, 53, 55, 56, 58, 60, 62};
        static const int P2[12] = {1, 3, 5, 7, 8, 10, 12, 14, 17, 19, 21, 23};
        for (int k = 0; k < 12; k++) {
            e->board[P1[k]] = 1;
            e->board[P2[k]] = 2;
        }
    }
    if (g->kind == LUDAX_REF_HASAMI_SHOGI) {
        /* App. C: each player fills the two rows on its side */
        for (int c = 0; c < 9; c++) {
            e->board[0 * 9 + c] = e->board[1 * 9 + c] = 2;
            e->board[7 * 9 + c] = e->board[8 * 9 + c] = 1;
        }
    }
    e->to_move = 1;
    e->status = LUDAX_REF_RUNNING;
    e->winner = -1;
    e->passes = 0;
    e->ply = 0;
    e->last_action = -1;
}

int ludax_ref_init(const ludax_ref_desc *d, ludax_ref_state *s, int64_t n)
{
    game_t g;
    int rc = resolve(d, &g);
    if (rc) return rc;
    if (n < 0 || (n > 0 && !state_ok(s))) return LUDAX_REF_E_INVALID;
    env_t e;
    for (int64_t i = 0; i < n; i++) {
        init_env(&g, &e);
        store_env(&g, s, i, &e);
    }
    return LUDAX_REF_OK;
}

/* ------------------------------------------------------------------ */
/* legal actions                                                       */
/* ------------------------------------------------------------------ */

static const int DIR8[8][2] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}, {1, 1}};

/* Number of opponent stones that a stone of `me` placed at (r, c) would
 * sandwich along direction (dr, dc): walk over the opponent's stones; the
 * first cell that is not the opponent's must be on the board and ours. */
static int flank_len(const game_t *g, const env_t *e, int r, int c, int dr, int dc, int me)
{
    int opp = 3 - me, k = 0;
    int rr = r + dr, cc = c + dc;
    while (on_board(g, rr, cc) && at(g, e, rr, cc) == opp) {
        k++;
        rr += dr;
        cc += dc;
    }
    if (k > 0 && on_board(g, rr, cc) && at(g, e, rr, cc) == me) return k;
    return 0;
}

static int reversi_placement_legal(const game_t *g, const env_t *e, int r, int c, int me)
{
    if (at(g, e, r, c) != 0) return 0;
    for (int d = 0; d < 8; d++)
        if (flank_len(g, e, r, c, DIR8[d][0], DIR8[d][1], me)) return 1;
    return 0;
}

/* ---- movement games (Wolf and Sheep, English Draughts) ---- */

static int is_move_game(const game_t *g)
{
    return g->kind == LUDAX_REF_WOLF_SHEEP || g->kind == LUDAX_REF_DRAUGHTS || g->kind == LUDAX_REF_HASAMI_SHOGI;
}

static const int ORTH4[4][2] = {{-1, 0}, {0, -1}, {0, 1}, {1, 0}};

/* Dai Hasami Shogi moves of the player to move: from each of its pieces,
 * along each row / column direction, a slide to every cell of the run of
 * empty cells next to it, or, if the neighbour is a piece (either
 * player's), a hop to the cell beyond it when that cell is empty. */
static int shogi_legal(const game_t *g, const env_t *e, uint8_t *m)
{
    int me = e->to_move, count = 0;
    for (int src = 0; src < g->cells; src++) {
        if (e->board[src] != me) continue;
        int r = src / g->W, c = src % g->W;
        for (int d = 0; d < 4; d++) {
            int dr = ORTH4[d][0], dc = ORTH4[d][1], k = 1;
            while (on_board(g, r + k * dr, c + k * dc) && at(g, e, r + k * dr, c + k * dc) == 0) {
                m[src * g->cells + (r + k * dr) * g->W + (c + k * dc)] = 1;
                count++;
                k++;
            }
            if (k == 1 && on_board(g, r + dr, c + dc) && on_board(g, r + 2 * dr, c + 2 * dc) &&
                at(g, e, r + 2 * dr, c + 2 * dc) == 0) {
                m[src * g->cells + (r + 2 * dr) * g->W + (c + 2 * dc)] = 1;
                count++;
            }
        }
    }
    return count;
}

/* May the piece with cell value v go in row direction dr (-1 up, +1 down)?
 * A Draughts king (bit 4) and the wolf go both ways; a pawn or a sheep only
 * forward: up for player 1, down for player 2. */
static int goes_both_ways(const game_t *g, int v)
{
    return g->kind == LUDAX_REF_DRAUGHTS ? (v & 4) != 0 : v == 2;
}

static int may_go(const game_t *g, int v, int dr)
{
    if (goes_both_ways(g, v)) return 1;
    return (v & 3) == 1 ? dr < 0 : dr > 0;
}

/* Destination of the move of the piece on `src` by `dist` (1 = step, 2 =
 * hop) cells in diagonal direction (dr, dc), or -1 if that move is not
 * allowed: the direction must suit the piece, the destination must be on
 * the board and empty, and a hop must pass over an opponent piece. */
static int move_dst(const game_t *g, const env_t *e, int src, int dr, int dc, int dist)
{
    int v = e->board[src], me = v & 3;
    if (!may_go(g, v, dr)) return -1;
    int r = src / g->W + dist * dr, c = src % g->W + dist * dc;
    if (!on_board(g, r, c) || at(g, e, r, c) != 0) return -1;
    if (dist == 2) {
        int over = at(g, e, src / g->W + dr, src % g->W + dc);
        if (over == 0 || (over & 3) != 3 - me) return -1;
    }
    return r * g->W + c;
}

static const int DIAG4[4][2] = {{-1, -1}, {-1, 1}, {1, -1}, {1, 1}};

/* Legal moves of the player to move: pieces of `me` (only the piece on
 * passes - 1 during a Draughts extra turn); the hops if there is any hop
 * (hop priority 0 over step priority 1, App. A listing), else the steps.
 * Marks m[src * cells + dst] and returns the number of moves. */
static int move_legal(const game_t *g, const env_t *e, uint8_t *m)
{
    if (g->kind == LUDAX_REF_HASAMI_SHOGI) return shogi_legal(g, e, m);
    int me = e->to_move;
    int only = (g->kind == LUDAX_REF_DRAUGHTS && e->passes > 0) ? e->passes - 1 : -1;
    int first = g->kind == LUDAX_REF_DRAUGHTS ? 2 : 1; /* Wolf and Sheep has no hops */
    for (int dist = first; dist >= 1; dist--) {
        int count = 0;
        for (int src = 0; src < g->cells; src++) {
            if (e->board[src] == 0 || (e->board[src] & 3) != me) continue;
            if (only >= 0 && src != only) continue;
            for (int d = 0; d < 4; d++) {
                int dst = move_dst(g, e, src, DIAG4[d][0], DIAG4[d][1], dist);
                if (dst >= 0) {
                    m[src * g->cells + dst] = 1;
                    count++;
                }
            }
        }
        if (count) return count;
    }
    return 0;
}

static void legal(const game_t *g, const env_t *e, uint8_t *m)
{
    memset(m, 0, (size_t)g->A);
    if (e->status != LUDAX_REF_RUNNING) return;
    int me = e->to_move;
    switch (g->kind) {
    case LUDAX_REF_TICTACTOE:
    case LUDAX_REF_HEX:
    case LUDAX_REF_GOMOKU:
    case LUDAX_REF_YAVALATH:
        for (int i = 0; i < g->cells; i++) m[i] = (e->board[i] == 0);
        break;
    case LUDAX_REF_PENTE: {
        int empty = 1;
        for (int i = 0; i < g->cells; i++) empty &= e->board[i] == 0;
        if (empty) { /* the first move goes to the exact centre */
            m[(g->H / 2) * g->W + g->W / 2] = 1;
            break;
        }
        for (int i = 0; i < g->cells; i++) m[i] = (e->board[i] == 0);
        break;
    }
    case LUDAX_REF_CONNECT_FOUR:
        /* an empty cell resting on the floor (bottom row) or on a piece */
        for (int r = 0; r < g->H; r++)
            for (int c = 0; c < g->W; c++)
                m[r * g->W + c] = at(g, e, r, c) == 0 && (r == g->H - 1 || at(g, e, r + 1, c) != 0);
        break;
    case LUDAX_REF_REVERSI: {
        int any = 0;
        for (int r = 0; r < g->H; r++)
            for (int c = 0; c < g->W; c++) {
                int ok = reversi_placement_legal(g, e, r, c, me);
                m[r * g->W + c] = (uint8_t)ok;
                any |= ok;
            }
        m[g->cells] = (uint8_t)!any; /* forced pass, and only then */
        break;
    }
    case LUDAX_REF_WOLF_SHEEP:
    case LUDAX_REF_DRAUGHTS:
    case LUDAX_REF_HASAMI_SHOGI:
        move_legal(g, e, m);
        break;
    }
}

int ludax_ref_legal_mask(const ludax_ref_desc *d, const ludax_ref_state *s, uint8_t *mask,
                         int64_t n)
{
    game_t g;
    int rc = resolve(d, &g);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!state_ok(s) || !mask))) return LUDAX_REF_E_INVALID;
    env_t e;
    for (int64_t i = 0; i < n; i++) {
        load_env(&g, s, i, &e);
        legal(&g, &e, mask + i * g.A);
    }
    return LUDAX_REF_OK;
}

/* ------------------------------------------------------------------ */
/* end rules                                                           */
/* ------------------------------------------------------------------ */

/* Does `who` own a maximal straight run whose length satisfies the rule
 * (length >= len, or exactly len)?  Full-board scan over the four line
 * orientations; a run is visited from its first cell only. */
static int has_line(const game_t *g, const env_t *e, int who, int len, int exact)
{
    static const int DIR4[4][2] = {{0, 1}, {1, 0}, {1, 1}, {1, -1}};
    for (int r = 0; r < g->H; r++)
        for (int c = 0; c < g->W; c++) {
            if (at(g, e, r, c) != who) continue;
            for (int d = 0; d < 4; d++) {
                int dr = DIR4[d][0], dc = DIR4[d][1];
                int pr = r - dr, pc = c - dc;
                if (on_board(g, pr, pc) && at(g, e, pr, pc) == who) continue; /* not a run start */
                int L = 0, rr = r, cc = c;
                while (on_board(g, rr, cc) && at(g, e, rr, cc) == who) {
                    L++;
                    rr += dr;
                    cc += dc;
                }
                if (exact ? (L == len) : (L >= len)) return 1;
            }
        }
    return 0;
}

/* Hex (App. C): a parallelogram of hexagons.  Neighbours of (r, c) are
 * (r-1,c) (r-1,c+1) (r,c-1) (r,c+1) (r+1,c-1) (r+1,c).  Player 1 joins the
 * top row to the bottom row, player 2 the left column to the right column.
 * Breadth-first search from every stone of `who` on its first side. */
static int hex_connected(const game_t *g, const env_t *e, int who)
{
    static const int NB[6][2] = {{-1, 0}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}};
    int N = g->H;
    uint8_t seen[MAX_CELLS];
    int queue[MAX_CELLS], qh = 0, qt = 0;
    memset(seen, 0, sizeof seen);
    for (int k = 0; k < N; k++) {
        int r = (who == 1) ? 0 : k, c = (who == 1) ? k : 0;
        int i = r * N + c;
        if (e->board[i] == who && !seen[i]) {
            seen[i] = 1;
            queue[qt++] = i;
        }
    }
    while (qh < qt) {
        int i = queue[qh++];
        int r = i / N, c = i % N;
        if ((who == 1 && r == N - 1) || (who == 2 && c == N - 1)) return 1;
        for (int d = 0; d < 6; d++) {
            int rr = r + NB[d][0], cc = c + NB[d][1];
            if (!on_board(g, rr, cc)) continue;
            int j = rr * N + cc;
            if (e->board[j] == who && !seen[j]) {
                seen[j] = 1;
                queue[qt++] = j;
            }
        }
    }
    return 0;
}

/* Yavalath geometry: row lengths, the first axial q of a row, and the cell
 * at axial (r, q) (-1 off the board). */
static int yav_len(const game_t *g, int r)
{
    int d = r - (g->S - 1);
    return g->H - (d < 0 ? -d : d);
}
static int yav_q0(const game_t *g, int r) { return r < g->S - 1 ? g->S - 1 - r : 0; }
static int yav_cell(const game_t *g, int r, int q)
{
    if (r < 0 || r >= g->H) return -1;
    int i = q - yav_q0(g, r);
    if (i < 0 || i >= yav_len(g, r)) return -1;
    int base = 0;
    for (int k = 0; k < r; k++) base += yav_len(g, k);
    return base + i;
}

/* Longest and shortest maximal straight runs of `who`: *longest = the
 * longest run, *has3 = some maximal run has exactly 3 stones.  Every cell
 * is visited as a potential run start in each of the three directions. */
static void yav_runs(const game_t *g, const env_t *e, int who, int *longest, int *has3)
{
    static const int DIR3[3][2] = {{0, 1}, {1, 0}, {1, -1}};
    *longest = 0;
    *has3 = 0;
    for (int r = 0; r < g->H; r++)
        for (int i = 0; i < yav_len(g, r); i++) {
            int q = i + yav_q0(g, r);
            if (e->board[yav_cell(g, r, q)] != who) continue;
            for (int d = 0; d < 3; d++) {
                int dr = DIR3[d][0], dq = DIR3[d][1];
                int prev = yav_cell(g, r - dr, q - dq);
                if (prev >= 0 && e->board[prev] == who) continue; /* not a run start */
                int L = 0, rr = r, qq = q, c;
                while ((c = yav_cell(g, rr, qq)) >= 0 && e->board[c] == who) {
                    L++;
                    rr += dr;
                    qq += dq;
                }
                if (L > *longest) *longest = L;
                if (L == 3) *has3 = 1;
            }
        }
}

static int board_full(const game_t *g, const env_t *e)
{
    for (int i = 0; i < g->cells; i++)
        if (e->board[i] == 0) return 0;
    return 1;
}

/* The mover's end rules, in the order the game lists them (Sec. 3.3).
 * Returns -1 if the game goes on, else the winner (0 = draw). */
static int end_rules(const game_t *g, const env_t *e, int me)
{
    switch (g->kind) {
    case LUDAX_REF_TICTACTOE:
        if (has_line(g, e, me, 3, 0)) return me;
        if (board_full(g, e)) return 0;
        return -1;
    case LUDAX_REF_CONNECT_FOUR:
        if (has_line(g, e, me, 4, 0)) return me;
        if (board_full(g, e)) return 0;
        return -1;
    case LUDAX_REF_GOMOKU:
        if (has_line(g, e, me, 5, 1)) return me;
        if (board_full(g, e)) return 0;
        return -1;
    case LUDAX_REF_HEX:
        if (hex_connected(g, e, me)) return me;
        return -1;
    case LUDAX_REF_YAVALATH: {
        /* four (or more) in a row wins; else three in a row loses */
        int longest, has3;
        yav_runs(g, e, me, &longest, &has3);
        if (longest >= 4) return me;
        if (has3) return 3 - me;
        if (board_full(g, e)) return 0;
        return -1;
    }
    case LUDAX_REF_PENTE: {
        /* five or more in a row, or 10 captured stones (5 pairs), wins */
        int pairs = me == 1 ? (e->passes & 15) : ((e->passes >> 4) & 15);
        if (has_line(g, e, me, 5, 0) || pairs >= 5) return me;
        if (board_full(g, e)) return 0;
        return -1;
    }
    case LUDAX_REF_REVERSI:
        if (e->passes >= 2) {
            int n1 = 0, n2 = 0;
            for (int i = 0; i < g->cells; i++) {
                n1 += e->board[i] == 1;
                n2 += e->board[i] == 2;
            }
            return n1 > n2 ? 1 : (n2 > n1 ? 2 : 0);
        }
        return -1;
    }
    return -1;
}

/* Consistency: the opponent of the mover can never hold a win after the
 * mover's ply (no captures in the line and connection games). */
static void check_opponent(const game_t *g, const env_t *e, int me)
{
    int opp = 3 - me;
    int bad = 0;
    switch (g->kind) {
    case LUDAX_REF_TICTACTOE: bad = has_line(g, e, opp, 3, 0); break;
    case LUDAX_REF_CONNECT_FOUR: bad = has_line(g, e, opp, 4, 0); break;
    case LUDAX_REF_GOMOKU: bad = has_line(g, e, opp, 5, 1); break;
    case LUDAX_REF_HEX: bad = hex_connected(g, e, opp); break;
    case LUDAX_REF_YAVALATH: {
        int longest, has3;
        yav_runs(g, e, opp, &longest, &has3);
        bad = longest >= 3;
        break;
    }
    case LUDAX_REF_PENTE: bad = has_line(g, e, opp, 5, 0); break;
    default: break;
    }
    if (bad) check_failed();
}

int ludax_ref_holds_win(const ludax_ref_desc *d, const int8_t *board, int who)
{
    game_t g;
    if (resolve(d, &g) || !board || (who != 1 && who != 2)) return -1;
    env_t e;
    memcpy(e.board, board, (size_t)g.cells);
    switch (g.kind) {
    case LUDAX_REF_TICTACTOE: return has_line(&g, &e, who, 3, 0);
    case LUDAX_REF_CONNECT_FOUR: return has_line(&g, &e, who, 4, 0);
    case LUDAX_REF_GOMOKU: return has_line(&g, &e, who, 5, 1);
    case LUDAX_REF_HEX: return hex_connected(&g, &e, who);
    case LUDAX_REF_YAVALATH: {
        int longest, has3;
        yav_runs(&g, &e, who, &longest, &has3);
        return longest >= 4;
    }
    case LUDAX_REF_PENTE: return has_line(&g, &e, who, 5, 0);
    default: return -1;
    }
}

/* ------------------------------------------------------------------ */
/* step                                                                */
/* ------------------------------------------------------------------ */

/* Dai Hasami Shogi captures after `me` moved a piece to dst: along each row
 * and column direction from dst, a run of one or more opponent pieces
 * closed by another piece of the mover's is removed; an opponent piece on
 * a corner is removed when both its neighbours are the mover's and one of
 * them is dst. */
static void shogi_captures(const game_t *g, env_t *e, int dst, int me)
{
    int opp = 3 - me, r = dst / g->W, c = dst % g->W;
    for (int d = 0; d < 4; d++) {
        int dr = ORTH4[d][0], dc = ORTH4[d][1], k = 1;
        while (on_board(g, r + k * dr, c + k * dc) && at(g, e, r + k * dr, c + k * dc) == opp) k++;
        if (k > 1 && on_board(g, r + k * dr, c + k * dc) && at(g, e, r + k * dr, c + k * dc) == me)
            for (int j = 1; j < k; j++) e->board[(r + j * dr) * g->W + (c + j * dc)] = 0;
    }
    static const int CORNER[4][2] = {{0, 0}, {0, 8}, {8, 0}, {8, 8}};
    for (int q = 0; q < 4; q++) {
        int cr = CORNER[q][0], cc = CORNER[q][1];
        int vr = cr == 0 ? 1 : cr - 1, hc = cc == 0 ? 1 : cc - 1; /* its column and row neighbours */
        int v = vr * g->W + cc, h = cr * g->W + hc;
        if (at(g, e, cr, cc) == opp && e->board[v] == me && e->board[h] == me && (dst == v || dst == h))
            e->board[cr * g->W + cc] = 0;
    }
}

/* A legal move of a movement game and its effects (Sec. 3.2; the order of
 * the App. A Draughts listing: move and capture, then promotion, then the
 * extra-turn test).  Returns the player who moves next. */
static int apply_move(const game_t *g, env_t *e, int a, int me)
{
    int src = a / g->cells, dst = a % g->cells;
    int v = e->board[src];
    int rs = src / g->W, cs = src % g->W, rd = dst / g->W, cd = dst % g->W;
    e->board[src] = 0;
    e->board[dst] = (int8_t)v;
    e->passes = 0;
    if (g->kind == LUDAX_REF_HASAMI_SHOGI) { /* slides and hops only move the piece */
        shogi_captures(g, e, dst, me);
        return 3 - me;
    }
    int hop = rd - rs == 2 || rs - rd == 2;
    if (hop) e->board[((rs + rd) / 2) * g->W + (cs + cd) / 2] = 0; /* the hopped piece is captured */
    if (g->kind != LUDAX_REF_DRAUGHTS) return 3 - me;
    if (!(v & 4) && rd == (me == 1 ? 0 : g->H - 1)) e->board[dst] = (int8_t)(v | 4); /* promotion */
    if (hop)
        for (int d = 0; d < 4; d++)
            if (move_dst(g, e, dst, DIAG4[d][0], DIAG4[d][1], 2) >= 0) {
                e->passes = (int8_t)(dst + 1); /* extra turn for the same piece */
                return me;
            }
    return 3 - me;
}

/* Dai Hasami Shogi's win: five of `me`'s pieces in a row or a column, none
 * of them on me's two start rows. */
static int shogi_five(const game_t *g, const env_t *e, int me)
{
    int lo = me == 1 ? 0 : 2, hi = me == 1 ? 6 : 8; /* rows outside the start rows */
    for (int r = lo; r <= hi; r++)
        for (int c = 0; c < g->W; c++) {
            int row = c + 5 <= g->W, col = r + 4 <= hi;
            for (int k = 0; k < 5 && (row || col); k++) {
                if (row && !(on_board(g, r, c + k) && at(g, e, r, c + k) == me)) row = 0;
                if (col && at(g, e, r + k, c) != me) col = 0;
            }
            if (row || col) return 1;
        }
    return 0;
}

/* End rules of a movement game after the mover's ply, `next` being the
 * player to move next: the wolf on the bottom row wins (Wolf and Sheep),
 * then the mover wins if `next` has no legal action. */
static int move_end_rules(const game_t *g, const env_t *e, int me, int next)
{
    if (g->kind == LUDAX_REF_WOLF_SHEEP && me == 2)
        for (int c = 0; c < g->W; c++)
            if (at(g, e, g->H - 1, c) == 2) return 2;
    if (g->kind == LUDAX_REF_HASAMI_SHOGI && shogi_five(g, e, me)) return me;
    env_t t = *e;
    t.to_move = next;
    uint8_t m[MAX_ACTIONS];
    memset(m, 0, (size_t)g->A);
    if (move_legal(g, &t, m) == 0) return me;
    return -1;
}

static void step_env(const game_t *g, env_t *e, int32_t a, int8_t rew[2], uint8_t *term)
{
    rew[0] = rew[1] = 0;
    if (e->status != LUDAX_REF_RUNNING) { /* stepping an ended env: no-op */
        *term = 1;
        return;
    }
    uint8_t m[MAX_ACTIONS];
    legal(g, e, m);
    if (a < 0 || a >= g->A || !m[a]) { /* illegal: flag it, change nothing else */
        e->status = LUDAX_REF_ILLEGAL;
        *term = 1;
        return;
    }
    int me = e->to_move, next = 3 - me;
    if (is_move_game(g)) {
        next = apply_move(g, e, a, me);
    } else if (g->kind == LUDAX_REF_REVERSI && a == g->cells) {
        e->passes += 1;
    } else {
        int r = a / g->W, c = a % g->W;
        if (g->kind == LUDAX_REF_REVERSI) {
            /* find every sandwiched line first, then flip them all */
            int len[8];
            for (int d = 0; d < 8; d++) len[d] = flank_len(g, e, r, c, DIR8[d][0], DIR8[d][1], me);
            for (int d = 0; d < 8; d++)
                for (int k = 1; k <= len[d]; k++)
                    e->board[(r + k * DIR8[d][0]) * g->W + (c + k * DIR8[d][1])] = (int8_t)me;
            e->passes = 0;
        }
        e->board[a] = (int8_t)me;
        if (g->kind == LUDAX_REF_PENTE) {
            /* custodial capture of exactly two: in each of the 8 directions,
             * two opponent stones and then one of the mover's */
            int opp = 3 - me, pairs = 0;
            for (int d = 0; d < 8; d++) {
                int dr = DIR8[d][0], dc = DIR8[d][1];
                int r1 = r + dr, c1 = c + dc, r2 = r + 2 * dr, c2 = c + 2 * dc, r3 = r + 3 * dr, c3 = c + 3 * dc;
                if (on_board(g, r3, c3) && at(g, e, r1, c1) == opp && at(g, e, r2, c2) == opp &&
                    at(g, e, r3, c3) == me) {
                    e->board[r1 * g->W + c1] = 0;
                    e->board[r2 * g->W + c2] = 0;
                    pairs++;
                }
            }
            int lo = e->passes & 15, hi = (e->passes >> 4) & 15;
            if (me == 1) lo += pairs;
            else hi += pairs;
            e->passes = (int8_t)(lo | (hi << 4));
        }
    }
    e->ply += 1;
    e->last_action = a;

    int w = is_move_game(g) ? move_end_rules(g, e, me, next) : end_rules(g, e, me);
    if (g_checks) check_opponent(g, e, me);
    if (w >= 0) {
        e->status = LUDAX_REF_TERMINAL;
        e->winner = w;
        if (w == 1) { rew[0] = 1; rew[1] = -1; }
        if (w == 2) { rew[0] = -1; rew[1] = 1; }
    } else {
        e->to_move = next;
        if (e->ply >= g->max_plies) {
            e->status = LUDAX_REF_TRUNCATED;
            e->winner = -1;
        }
    }
    *term = (uint8_t)(e->status != LUDAX_REF_RUNNING);
}

int ludax_ref_step(const ludax_ref_desc *d, ludax_ref_state *s, const int32_t *action,
                   int8_t *reward, uint8_t *terminal, uint8_t *next_mask, int64_t n)
{
    game_t g;
    int rc = resolve(d, &g);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!state_ok(s) || !action || !reward || !terminal)))
        return LUDAX_REF_E_INVALID;
    env_t e;
    for (int64_t i = 0; i < n; i++) {
        load_env(&g, s, i, &e);
        step_env(&g, &e, action[i], reward + 2 * i, terminal + i);
        store_env(&g, s, i, &e);
        if (next_mask) legal(&g, &e, next_mask + i * g.A);
    }
    return LUDAX_REF_OK;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 and the playout                                       */
/* ------------------------------------------------------------------ */

void ludax_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    /* Salmon et al. SC'11: each round multiplies counter words 0 and 2 by
     * the two Philox multipliers, and the new counter is
     * (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
     * between rounds the key is bumped by the two Weyl constants. */
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

uint32_t ludax_ref_draw(uint64_t seed, int64_t game_id, int32_t ply)
{
    /* counter = (ply / 4, low and high words of the game id, 0),
     * key = (low and high words of the seed); word ply % 4 of the block. */
    uint64_t gid = (uint64_t)game_id;
    uint32_t ctr[4] = {(uint32_t)ply >> 2, (uint32_t)gid, (uint32_t)(gid >> 32), 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    ludax_ref_philox4x32_10(ctr, key, out);
    return out[(uint32_t)ply & 3u];
}

typedef struct {
    int64_t steps, w1, w2, draws;
} tally_t;

static void playout_env(const game_t *g, env_t *e, uint64_t seed, int64_t gid, int8_t rew[2],
                        uint8_t *term, tally_t *t)
{
    rew[0] = rew[1] = 0;
    uint8_t m[MAX_ACTIONS];
    while (e->status == LUDAX_REF_RUNNING) {
        legal(g, e, m);
        int nlegal = 0;
        for (int a = 0; a < g->A; a++) nlegal += m[a];
        if (nlegal == 0) { /* only on a hand-made, unreachable state */
            e->status = LUDAX_REF_ILLEGAL;
            break;
        }
        /* uniform choice among the legal actions: multiply-shift of one
         * 32-bit Philox word, then the k-th legal action in index order */
        uint32_t w = ludax_ref_draw(seed, gid, e->ply);
        int k = (int)(((uint64_t)w * (uint64_t)nlegal) >> 32);
        int a = -1;
        for (int i = 0; i < g->A; i++)
            if (m[i]) {
                if (k == 0) {
                    a = i;
                    break;
                }
                k--;
            }
        uint8_t tt;
        step_env(g, e, a, rew, &tt);
        t->steps++;
    }
    *term = 1;
    if (e->status == LUDAX_REF_TERMINAL) {
        if (e->winner == 1) t->w1++;
        else if (e->winner == 2) t->w2++;
        else if (e->winner == 0) t->draws++;
    }
}

typedef struct {
    const game_t *g;
    ludax_ref_state *s;
    uint64_t seed;
    int64_t base;
    const int64_t *gid;
    int8_t *reward;
    uint8_t *terminal;
    int64_t lo, hi;
    tally_t t;
} job_t;

static void *playout_range(void *arg)
{
    job_t *j = (job_t *)arg;
    env_t e;
    memset(&j->t, 0, sizeof j->t);
    for (int64_t i = j->lo; i < j->hi; i++) {
        load_env(j->g, j->s, i, &e);
        int was_running = e.status == LUDAX_REF_RUNNING;
        int64_t gid = j->gid ? j->gid[i] : j->base + i;
        tally_t t = {0, 0, 0, 0};
        playout_env(j->g, &e, j->seed, gid, j->reward + 2 * i, j->terminal + i, &t);
        /* outcomes are counted only for games that ended inside this call */
        if (!was_running) t.w1 = t.w2 = t.draws = 0;
        j->t.steps += t.steps;
        j->t.w1 += t.w1;
        j->t.w2 += t.w2;
        j->t.draws += t.draws;
        store_env(j->g, j->s, i, &e);
    }
    return NULL;
}

int ludax_ref_playout(const ludax_ref_desc *d, ludax_ref_state *s, uint64_t seed,
                      int64_t game_id_base, const int64_t *game_id, int8_t *reward,
                      uint8_t *terminal, int64_t *stats, int64_t n, int threads)
{
    game_t g;
    int rc = resolve(d, &g);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!state_ok(s) || !reward || !terminal))) return LUDAX_REF_E_INVALID;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if (threads > n) threads = (int)(n > 0 ? n : 1);
    job_t jobs[256];
    pthread_t tid[256];
    for (int k = 0; k < threads; k++) {
        jobs[k].g = &g;
        jobs[k].s = s;
        jobs[k].seed = seed;
        jobs[k].base = game_id_base;
        jobs[k].gid = game_id;
        jobs[k].reward = reward;
        jobs[k].terminal = terminal;
        jobs[k].lo = n * k / threads;
        jobs[k].hi = n * (k + 1) / threads;
    }
    if (threads == 1) {
        playout_range(&jobs[0]);
    } else {
        for (int k = 0; k < threads; k++) pthread_create(&tid[k], NULL, playout_range, &jobs[k]);
        for (int k = 0; k < threads; k++) pthread_join(tid[k], NULL);
    }
    if (stats)
        for (int k = 0; k < threads; k++) {
            stats[0] += jobs[k].t.steps;
            stats[1] += jobs[k].t.w1;
            stats[2] += jobs[k].t.w2;
            stats[3] += jobs[k].t.draws;
        }
    return LUDAX_REF_OK;
}

/* ------------------------------------------------------------------ */
/* enumeration helpers                                                 */
/* ------------------------------------------------------------------ */

static int64_t perft_rec(const game_t *g, const env_t *e, int depth)
{
    if (depth == 0) return 1;
    if (e->status != LUDAX_REF_RUNNING) return 0;
    uint8_t m[MAX_ACTIONS];
    legal(g, e, m);
    int64_t total = 0;
    for (int a = 0; a < g->A; a++) {
        if (!m[a]) continue;
        env_t c = *e;
        int8_t rew[2];
        uint8_t t;
        step_env(g, &c, a, rew, &t);
        total += perft_rec(g, &c, depth - 1);
    }
    return total;
}

int64_t ludax_ref_perft(const ludax_ref_desc *d, const ludax_ref_state *s, int depth)
{
    game_t g;
    if (resolve(d, &g) || !state_ok(s) || depth < 0) return -1;
    env_t e;
    load_env(&g, s, 0, &e);
    return perft_rec(&g, &e, depth);
}

/* As perft_rec, but a ply after which the same player moves again (an
 * extra turn) does not use up a level. */
static int64_t perft_turns_rec(const game_t *g, const env_t *e, int depth)
{
    if (depth == 0) return 1;
    if (e->status != LUDAX_REF_RUNNING) return 0;
    uint8_t m[MAX_ACTIONS];
    legal(g, e, m);
    int64_t total = 0;
    for (int a = 0; a < g->A; a++) {
        if (!m[a]) continue;
        env_t c = *e;
        int8_t rew[2];
        uint8_t t;
        step_env(g, &c, a, rew, &t);
        int again = c.status == LUDAX_REF_RUNNING && c.to_move == e->to_move;
        total += perft_turns_rec(g, &c, again ? depth : depth - 1);
    }
    return total;
}

int64_t ludax_ref_perft_turns(const ludax_ref_desc *d, const ludax_ref_state *s, int depth)
{
    game_t g;
    if (resolve(d, &g) || !state_ok(s) || depth < 0) return -1;
    env_t e;
    load_env(&g, s, 0, &e);
    return perft_turns_rec(&g, &e, depth);
}

static int64_t games_rec(const game_t *g, const env_t *e, int64_t *tab, int max_len,
                         int64_t *trunc)
{
    if (e->status != LUDAX_REF_RUNNING) {
        if (e->status == LUDAX_REF_TERMINAL && e->ply <= max_len && e->winner >= 0)
            tab[e->ply * 3 + e->winner]++;
        else if (trunc)
            (*trunc)++;
        return 1;
    }
    uint8_t m[MAX_ACTIONS];
    legal(g, e, m);
    int64_t total = 0;
    for (int a = 0; a < g->A; a++) {
        if (!m[a]) continue;
        env_t c = *e;
        int8_t rew[2];
        uint8_t t;
        step_env(g, &c, a, rew, &t);
        total += games_rec(g, &c, tab, max_len, trunc);
    }
    return total;
}

int64_t ludax_ref_count_games(const ludax_ref_desc *d, const ludax_ref_state *s,
                              int64_t *by_len_winner, int max_len, int64_t *truncated)
{
    game_t g;
    if (resolve(d, &g) || !state_ok(s) || !by_len_winner || max_len < 0) return -1;
    env_t e;
    load_env(&g, s, 0, &e);
    return games_rec(&g, &e, by_len_winner, max_len, truncated);
}
