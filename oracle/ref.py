"""ctypes wrapper of the plain CPU oracle (``oracle/ludax_ref.c``).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
leg of the benchmark use it to check the GPU library; the GPU library never
imports it.  It works on numpy arrays in host memory.  If the shared object
is missing it is compiled once with gcc (the oracle is plain C11).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ludax_ref.c")
LIB = os.path.join(HERE, "libludax_ref.so")

TICTACTOE, CONNECT_FOUR, HEX, REVERSI, GOMOKU, YAVALATH, PENTE, WOLF_SHEEP, DRAUGHTS, HASAMI_SHOGI = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10
RUNNING, TERMINAL, TRUNCATED, ILLEGAL = 0, 1, 2, 3

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/libludax_ref.so``."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
        os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "ludax_ref.h"))
    ):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp, SRC,
             "-lpthread"]
        )
        os.replace(tmp, LIB)
    return LIB


class _Desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("max_plies", ctypes.c_int32)]


class _State(ctypes.Structure):
    _fields_ = [("board", ctypes.c_void_p), ("to_move", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("winner", ctypes.c_void_p),
                ("passes", ctypes.c_void_p), ("ply", ctypes.c_void_p),
                ("last_action", ctypes.c_void_p)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(LIB)
            P = ctypes.POINTER
            L.ludax_ref_info.argtypes = [P(_Desc), P(ctypes.c_int32), P(ctypes.c_int32),
                                         P(ctypes.c_int32)]
            L.ludax_ref_init.argtypes = [P(_Desc), P(_State), ctypes.c_int64]
            L.ludax_ref_legal_mask.argtypes = [P(_Desc), P(_State), ctypes.c_void_p,
                                               ctypes.c_int64]
            L.ludax_ref_step.argtypes = [P(_Desc), P(_State), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
            L.ludax_ref_playout.argtypes = [P(_Desc), P(_State), ctypes.c_uint64, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
            L.ludax_ref_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p]
            L.ludax_ref_philox4x32_10.restype = None
            L.ludax_ref_draw.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32]
            L.ludax_ref_draw.restype = ctypes.c_uint32
            L.ludax_ref_perft.argtypes = [P(_Desc), P(_State), ctypes.c_int]
            L.ludax_ref_perft.restype = ctypes.c_int64
            L.ludax_ref_perft_turns.argtypes = [P(_Desc), P(_State), ctypes.c_int]
            L.ludax_ref_perft_turns.restype = ctypes.c_int64
            L.ludax_ref_count_games.argtypes = [P(_Desc), P(_State), ctypes.c_void_p, ctypes.c_int,
                                                ctypes.c_void_p]
            L.ludax_ref_count_games.restype = ctypes.c_int64
            L.ludax_ref_holds_win.argtypes = [P(_Desc), ctypes.c_void_p, ctypes.c_int]
            L.ludax_ref_holds_win.restype = ctypes.c_int
            L.ludax_ref_set_checks.argtypes = [ctypes.c_int]
            L.ludax_ref_set_checks.restype = None
            L.ludax_ref_check_failures.argtypes = []
            L.ludax_ref_check_failures.restype = ctypes.c_int64
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        raise OracleError("oracle returned %d" % rc)


@dataclass
class Game:
    kind: int
    rows: int
    cols: int
    max_plies: int = 0

    def desc(self) -> _Desc:
        return _Desc(self.kind, self.rows, self.cols, self.max_plies)

    def info(self):
        cells, A, mp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        rc = lib().ludax_ref_info(ctypes.byref(self.desc()), ctypes.byref(cells), ctypes.byref(A),
                                  ctypes.byref(mp))
        _check(rc)
        return cells.value, A.value, mp.value

    @property
    def cells(self):
        return self.info()[0]

    @property
    def num_actions(self):
        return self.info()[1]


class State:
    """Host SoA batch state (numpy)."""

    FIELDS = ("board", "to_move", "status", "winner", "passes", "ply", "last_action")

    def __init__(self, n: int, cells: int):
        self.n, self.cells = n, cells
        self.board = np.zeros((n, cells), np.int8)
        self.to_move = np.zeros(n, np.int8)
        self.status = np.zeros(n, np.int8)
        self.winner = np.zeros(n, np.int8)
        self.passes = np.zeros(n, np.int8)
        self.ply = np.zeros(n, np.int16)
        self.last_action = np.zeros(n, np.int16)

    def c(self) -> _State:
        return _State(*[_ptr(getattr(self, f)) for f in self.FIELDS])

    def copy(self) -> "State":
        s = State(self.n, self.cells)
        for f in self.FIELDS:
            setattr(s, f, getattr(self, f).copy())
        return s

    def subset(self, idx) -> "State":
        idx = np.asarray(idx)
        s = State(len(idx), self.cells)
        for f in self.FIELDS:
            setattr(s, f, np.ascontiguousarray(getattr(self, f)[idx]))
        return s

    def as_dict(self):
        return {f: getattr(self, f) for f in self.FIELDS}


def init(game: Game, n: int) -> State:
    s = State(n, game.cells)
    _check(lib().ludax_ref_init(ctypes.byref(game.desc()), ctypes.byref(s.c()), n))
    return s


def legal_mask(game: Game, s: State) -> np.ndarray:
    m = np.zeros((s.n, game.num_actions), np.uint8)
    _check(lib().ludax_ref_legal_mask(ctypes.byref(game.desc()), ctypes.byref(s.c()), _ptr(m), s.n))
    return m


def step(game: Game, s: State, action, want_mask: bool = True):
    a = np.ascontiguousarray(np.asarray(action, dtype=np.int32))
    assert a.shape == (s.n,)
    rew = np.zeros((s.n, 2), np.int8)
    term = np.zeros(s.n, np.uint8)
    nm = np.zeros((s.n, game.num_actions), np.uint8) if want_mask else None
    _check(lib().ludax_ref_step(ctypes.byref(game.desc()), ctypes.byref(s.c()), _ptr(a), _ptr(rew),
                                _ptr(term), _ptr(nm) if nm is not None else None, s.n))
    return rew, term, nm


def playout(game: Game, s: State, seed: int, game_id_base: int = 0, game_id=None,
            threads: int = 1):
    rew = np.zeros((s.n, 2), np.int8)
    term = np.zeros(s.n, np.uint8)
    stats = np.zeros(4, np.int64)
    gid = None
    if game_id is not None:
        gid = np.ascontiguousarray(np.asarray(game_id, dtype=np.int64))
        assert gid.shape == (s.n,)
    _check(lib().ludax_ref_playout(ctypes.byref(game.desc()), ctypes.byref(s.c()),
                                   ctypes.c_uint64(seed & (2**64 - 1)), game_id_base,
                                   _ptr(gid) if gid is not None else None, _ptr(rew), _ptr(term),
                                   _ptr(stats), s.n, threads))
    return rew, term, stats


def philox(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, np.uint32)
    lib().ludax_ref_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(seed: int, game_id: int, ply: int) -> int:
    return lib().ludax_ref_draw(ctypes.c_uint64(seed & (2**64 - 1)), game_id, ply)


def perft(game: Game, s: State, depth: int) -> int:
    return lib().ludax_ref_perft(ctypes.byref(game.desc()), ctypes.byref(s.c()), depth)


def perft_turns(game: Game, s: State, depth: int) -> int:
    return lib().ludax_ref_perft_turns(ctypes.byref(game.desc()), ctypes.byref(s.c()), depth)


def count_games(game: Game, s: State, max_len: int):
    tab = np.zeros((max_len + 1, 3), np.int64)
    trunc = ctypes.c_int64(0)
    total = lib().ludax_ref_count_games(ctypes.byref(game.desc()), ctypes.byref(s.c()), _ptr(tab),
                                        max_len, ctypes.byref(trunc))
    return total, tab, trunc.value


def holds_win(game: Game, board, who: int) -> int:
    b = np.ascontiguousarray(np.asarray(board, dtype=np.int8).reshape(-1))
    assert b.size == game.cells
    return lib().ludax_ref_holds_win(ctypes.byref(game.desc()), _ptr(b), who)


def set_checks(on: bool):
    lib().ludax_ref_set_checks(1 if on else 0)


def check_failures() -> int:
    return lib().ludax_ref_check_failures()
