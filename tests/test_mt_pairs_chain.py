"""The generated scan of one group of 10 MT19937 jump coefficients
(paper_1307_5869_amd/csrc/mt_pairs.inc): it is what gen_mt_pairs.py writes,
and, run as the goto chain it is, it applies every set coefficient of each of
the 1024 bit patterns exactly once (as pairs and at most one single) and no
other coefficient.  Host only."""
import os
import re
import subprocess
import sys

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1307_5869_amd", "csrc")


def read_inc():
    return open(os.path.join(CSRC, "mt_pairs.inc")).read()


def test_inc_is_the_generator_output():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_mt_pairs.py")], capture_output=True, text=True,
                         check=True).stdout
    assert out.strip() == read_inc().strip()


def parse(text):
    """statements in order: (label or None, kind, args); kinds: test (bit, negate, target), pair, one, goto"""
    stmts = []
    for line in text.splitlines():
        line = line.strip()
        if not line or line.startswith("//"):
            continue
        label = None
        m = re.match(r"^(mt_\w+):\s*(.*)$", line)
        if m:
            label, line = m.group(1), m.group(2)
        for part in re.findall(r"if \(!?MT_BIT\(\d+\)\) goto \w+;|if \(MT_BIT\(\d+\)\) \{[^}]*\}|MT_PAIR\(\d+, \d+\);|"
                               r"MT_ONE\(\d+\);|goto \w+;|;", line):
            stmts.append((label, part))
            label = None
        if label is not None:
            stmts.append((label, ";"))
    return stmts


def run(stmts, bits):
    labels = {lab: i for i, (lab, _) in enumerate(stmts) if lab}
    applied, pc, steps = [], 0, 0
    while pc < len(stmts):
        steps += 1
        assert steps < 1000
        _, s = stmts[pc]
        m = re.match(r"if \((!?)MT_BIT\((\d+)\)\) goto (\w+);", s)
        if m:
            taken = bool(bits >> int(m.group(2)) & 1) != (m.group(1) == "!")
            pc = labels[m.group(3)] if taken else pc + 1
            continue
        m = re.match(r"MT_PAIR\((\d+), (\d+)\);", s)
        if m:
            applied += [int(m.group(1)), int(m.group(2))]
        m = re.match(r"MT_ONE\((\d+)\);", s)
        if m:
            applied.append(int(m.group(1)))
        m = re.match(r"goto (\w+);", s)
        if m:
            pc = labels[m.group(1)]
            continue
        pc += 1
    return applied


def test_chain_applies_each_set_coefficient_once():
    stmts = parse(read_inc())
    assert any(lab == "mt_END" for lab, _ in stmts)
    for bits in range(1024):
        got = run(stmts, bits)
        want = [u for u in range(10) if bits >> u & 1]
        assert sorted(got) == want, (bits, got)
