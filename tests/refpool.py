"""Oracle references for the full-size parity tests, computed on host threads
(the oracle's C calls release the interpreter lock), and MT19937 jump
polynomials built once from the oracle's own products mod phi."""
import concurrent.futures as cf
import os

import numpy as np

MT = 0


def workers():
    return max(1, min(16, os.cpu_count() or 1))


def pmap(fn, items):
    """fn over items on a thread pool, results in order."""
    with cf.ThreadPoolExecutor(max_workers=workers()) as ex:
        return list(ex.map(fn, items))


class MtLadder:
    """x^(2^(e + b)) mod phi for b < nbits, from one oracle Frobenius power
    and repeated squaring (the oracle's product mod phi)."""

    def __init__(self, oracle, e, nbits):
        self.O = oracle
        oracle.mt_charpoly()            # phi once, before any thread uses it
        lad = [oracle.mt_frobenius(e)]
        for _ in range(1, nbits):
            lad.append(oracle.mt_poly_mulmod(lad[-1], lad[-1]))
        self.lad = lad

    def poly(self, m):
        """x^(m * 2^e) mod phi for m < 2^nbits."""
        g = 1
        for b in range(len(self.lad)):
            if (m >> b) & 1:
                g = self.O.mt_poly_mulmod(g, self.lad[b])
        return g

    def jump(self, base, m):
        """base (at a block boundary) jumped m * 2^e outputs."""
        st = base.copy()
        return self.O.mt_apply_poly(st, self.poly(m))


class StreamStarts:
    """Block-splitting start states from the default state, as the oracle
    defines them; MT19937 through the ladder (equal to the oracle's
    init_stream, checked on two ids when built)."""

    def __init__(self, oracle, gen):
        self.O, self.gen = oracle, gen
        self.mt = None
        if gen == MT:
            self.mt = MtLadder(oracle, oracle.block_log2(MT, 0), 64)
            self.base = oracle.init_default(MT)
            for sid in (1, 10**19 - 1):
                assert np.array_equal(self.mt.jump(self.base, sid), oracle.init_stream(MT, 0, sid))

    def __call__(self, sid):
        if self.mt is not None:
            return self.mt.jump(self.base, int(sid))
        return self.O.init_stream(self.gen, 0, int(sid))
