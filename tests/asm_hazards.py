"""Checks on the gfx950 assembly of the library's kernels (no GPU needed).

A matrix-core product needs a number of independent instructions ("wait
states") between its issue and the first read of its result by a vector
instruction, and a vector write needs a few before a product reads that
register.  The compiler inserts s_nop for these; the checks below look for
paths through a taken branch that leave fewer than the compiler itself uses on
straight-line code.  A taken branch counts as one wait state, as in the
compiler's own model.  Such a path once let a product's result be read before
the product finished (the loss saw a partial accumulator).
"""
import re

_LIST = re.compile(r'([av])\[(\d+):(\d+)\]$')
_ONE = re.compile(r'[av]\d+$')


def _regs(tok):
    tok = tok.strip(',')
    m = _LIST.match(tok)
    if m:
        return {m.group(1) + str(i) for i in range(int(m.group(2)), int(m.group(3)) + 1)}
    return {tok} if _ONE.match(tok) else set()


def _waits(ins):
    m = re.match(r's_nop (\d+)', ins)
    return int(m.group(1)) + 1 if m else 1


def parse(text):
    """Instructions (comments and directives dropped) and label positions."""
    ins, labels = [], {}
    for line in text.splitlines():
        s = line.split(';')[0].strip()
        if not s:
            continue
        if s.endswith(':'):
            labels[s[:-1]] = len(ins)
            continue
        if s.startswith('.'):
            continue
        ins.append(s)
    return ins, labels


def straight_line_needs(ins):
    """Wait states the compiler puts between a product and an immediate read of
    its result (s_nop N then the read), per product opcode: the largest seen."""
    need = {}
    for i, a in enumerate(ins):
        if not a.startswith('v_mfma'):
            continue
        # a run of s_nop (the compiler splits long waits: s_nop 15, s_nop 1)
        j, w = i + 1, 0
        while j < len(ins) and ins[j].startswith('s_nop'):
            w += _waits(ins[j])
            j += 1
        if w == 0 or j >= len(ins):
            continue
        c = ins[j]
        stores = c.startswith(('ds_write', 'global_store', 'buffer_store'))
        if (c.startswith('v_') and not c.startswith('v_mfma')) or stores:
            dst = _regs(a.split()[1])
            if any(_regs(x) & dst for x in c.split()[1 if stores else 2:]):
                op = a.split()[0]
                need[op] = max(need.get(op, 0), w)
    return need


def short_branch_paths(ins, labels, need, valu_need=2, window=30):
    """Taken-branch paths on which a product's result (or a product's operand
    written by a vector instruction) is read with too few wait states."""
    found = []
    for i, br in enumerate(ins):
        if not br.startswith(('s_cbranch', 's_branch')):
            continue
        tgt = br.split()[-1]
        if tgt not in labels:
            continue
        j0 = labels[tgt]
        # product issued before the branch, result read after the jump
        ws = 0
        for b in range(i - 1, max(-1, i - window), -1):
            t = ins[b]
            if t.startswith('v_mfma'):
                op = t.split()[0]
                dst = _regs(t.split()[1])
                w = ws + 1
                for c in range(j0, min(len(ins), j0 + window)):
                    u = ins[c]
                    ops = u.split()[1:]
                    stores = u.startswith(('ds_write', 'global_store', 'buffer_store'))
                    srcs = ops if stores else ops[1:]
                    if not u.startswith('v_mfma') and any(_regs(x) & dst for x in srcs):
                        if w < need.get(op, 11):
                            found.append((i, tgt, t, u, w))
                        break
                    if ops and not stores and u.startswith('v_'):
                        dst = dst - _regs(ops[0])   # overwritten before any read
                        if not dst:
                            break
                    w += _waits(u)
                    if w >= 32 or u.startswith(('s_cbranch', 's_branch', 's_endpgm')):
                        break
                break
            ws += _waits(t)
            if ws >= 32:
                break
        # vector write before the branch, product operand read after the jump
        ws = 0
        for b in range(i - 1, max(-1, i - 4), -1):
            t = ins[b]
            if t.startswith('v_') and not t.startswith(('v_mfma', 'v_cmp')):
                dst = _regs(t.split()[1])
                w = ws + 1
                for c in range(j0, min(len(ins), j0 + 4)):
                    u = ins[c]
                    if u.startswith('v_mfma') and any(_regs(x) & dst for x in u.split()[2:5]) and w < valu_need:
                        found.append((i, tgt, t, u, w))
                    w += _waits(u)
                    if w >= valu_need:
                        break
            ws += _waits(t)
    return found


def check(text, need=None):
    ins, labels = parse(text)
    need = dict(need or {})
    for op, n in straight_line_needs(ins).items():
        need[op] = max(need.get(op, 0), n)
    return short_branch_paths(ins, labels, need), need
