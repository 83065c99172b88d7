"""Build-time check of the generated gfx950 assembly: no loop that the
compiler structured as divergent (a loop exit accumulating an exec mask,
`s_andn2_b64 exec, exec, ...`) may contain a work-group barrier.  In such a
loop waves can reach the barrier a different number of times, which
deadlocks the work-group.  Usage: check_barriers.py file.s [--verbose];
exit status 1 when a loop is flagged.

Loop structure comes from the compiler's block annotations ("This Loop
Header", "in Loop: Header=", "Parent Loop"), which sit on the label line or
on the comment-only lines that follow it.  The block holding a loop's exec
exit can be laid out outside the loop's annotated blocks (before its header),
so an exec-mask exit also marks the loops whose headers it branches or falls
through to."""
import re, sys
from collections import defaultdict

LABEL = re.compile(r'^(?:\.L(BB\d+_\d+)|; %bb\.(\d+)):')


def annotation(body, i):
    """The label line's comment plus the comment-only lines after it."""
    text = [body[i]]
    k = i + 1
    while k < len(body) and body[k].strip().startswith(';') and not LABEL.match(body[k]):
        text.append(body[k])
        k += 1
    return ' '.join(text)


def check(asm, verbose=False):
    # data symbols (device globals) are labels too, with no function end
    objects = {m.group(1) for l in asm for m in [re.match(r'^\s*\.type\s+(\S+),\s*@object', l)]
               if m}
    starts = [i for i, l in enumerate(asm)
              if re.match(r'^_Z\S+:', l) and l.split(':')[0] not in objects]
    flagged = []
    for si in starts:
        sym = asm[si].split(':')[0]
        end = next(i for i in range(si + 1, len(asm)) if asm[i].startswith('.Lfunc_end'))
        body = asm[si:end]
        parents = {}          # loop header -> enclosing loop headers
        cur_loops = []        # loops of the current block, innermost first
        has_bar = defaultdict(bool)
        div = defaultdict(bool)
        exits = []            # labels reached from an exec-mask exit
        for i, l in enumerate(body):
            m = LABEL.match(l)
            if m:
                name = m.group(1)
                ann = annotation(body, i)
                ps = re.findall(r'Parent Loop (BB\d+_\d+)', ann)
                if name and re.search(r'This (?:Inner )?Loop Header', ann):
                    # innermost enclosing loop first
                    parents[name] = sorted(set(ps), key=lambda h: -ps.index(h))
                    cur_loops = [name] + parents[name]
                else:
                    hm = re.search(r'in Loop: Header=(BB\d+_\d+)', ann)
                    cur_loops = ([hm.group(1)] + parents.get(hm.group(1), [])) if hm else []
            t = l.strip()
            if t.startswith('s_barrier'):
                for h in cur_loops:
                    has_bar[h] = True
            if 's_andn2_b64 exec, exec' in t:
                for h in cur_loops[:1]:
                    div[h] = True
                k = i + 1
                while k < len(body) and not LABEL.match(body[k]):
                    bm = re.match(r'\s*s_cbranch_exec(?:nz|z)\s+\.L(BB\d+_\d+)', body[k])
                    if bm:
                        exits.append(bm.group(1))
                    k += 1
                if k < len(body):
                    fm = LABEL.match(body[k])
                    if fm and fm.group(1):
                        exits.append(fm.group(1))
        for h in exits:
            if h in parents:
                div[h] = True
        for h in div:
            if has_bar[h]:
                flagged.append((sym, h))
                if verbose:
                    print('DIVERGENT LOOP WITH BARRIER', sym[:100], h)
    return len(starts), flagged


if __name__ == '__main__':
    asm = open(sys.argv[1]).read().split('\n')
    total, flagged = check(asm, len(sys.argv) > 2)
    print('kernels checked', total, 'flagged loops', len(flagged), 'kernels',
          len(set(s for s, _ in flagged)))
    sys.exit(1 if flagged else 0)
