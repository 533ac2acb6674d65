"""Vector-memory instruction counts along the control-flow paths of a gfx9
kernel's assembly: basic blocks from labels, branches and fall-through."""
import re

VM = re.compile(r'^\s+(global_|buffer_|scratch_|flat_)')
BR = re.compile(r'\bs_(cbranch_\w+|branch)\s+(\.LBB\w+)')


def kernels(text):
    """{symbol: [lines]} of every kernel body in an assembly file."""
    out, cur, name = {}, None, None
    for l in text.splitlines():
        m = re.match(r'^(_Z\w+):', l)
        if m:
            name, cur = m.group(1), []
        if cur is not None:
            cur.append(l)
            if re.search(r'\bs_endpgm\b', l):
                out[name] = cur
                cur = None
    return out


def path_counts(L, start, target):
    """(min, max) number of vector-memory instructions executed on the paths
    from line index start to line index target (max capped at 999)."""
    lead, lab = {0, start, target}, {}
    for i, l in enumerate(L):
        m = re.match(r'^(\.LBB\w+):', l)
        if m:
            lab[m.group(1)] = i
            lead.add(i)
        if re.search(r'\bs_(cbranch_\w+|branch|endpgm)\b', l):
            lead.add(i + 1)
    lead = sorted(x for x in lead if x < len(L))
    end = dict(zip(lead, lead[1:] + [len(L)]))

    def succ(a):
        e = end[a]
        last = max((i for i in range(a, e) if L[i].strip() and not L[i].strip().startswith(';')), default=None)
        if last is not None:
            m = BR.search(L[last])
            if m:
                return [lab[m.group(2)]] + ([e] if m.group(1) != 'branch' and e < len(L) else [])
            if re.search(r'\bs_endpgm\b', L[last]):
                return []
        return [e] if e < len(L) else []

    def cnt(a):
        return sum(1 for i in range(a, end[a]) if VM.match(L[i]))

    lo, hi = {start: 0}, {start: 0}
    for _ in range(len(lead) + 2):
        ch = False
        for a in list(lo):
            if a == target:
                continue
            for b in succ(a):
                v = lo[a] + cnt(a)
                if v < lo.get(b, 10 ** 9):
                    lo[b] = v
                    ch = True
        if not ch:
            break
    for _ in range(80):
        ch = False
        for a in list(hi):
            if a == target:
                continue
            for b in succ(a):
                v = min(hi[a] + cnt(a), 999)
                if v > hi.get(b, -1):
                    hi[b] = v
                    ch = True
        if not ch:
            break
    return lo.get(target), hi.get(target)
