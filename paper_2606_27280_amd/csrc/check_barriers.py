"""Build-time check of the generated gfx950 assembly: no loop that the
compiler structured as divergent (a loop exit accumulating an exec mask,
`s_andn2_b64 exec, exec, ...`) may contain a work-group barrier.  In such a
loop waves can reach the barrier a different number of times, which
deadlocks the work-group.  Usage: check_barriers.py file.s [--verbose];
exit status 1 when a loop is flagged."""
import re, sys
from collections import defaultdict
asm = open(sys.argv[1]).read().split('\n')
starts = [i for i, l in enumerate(asm) if re.match(r'^_Z\S+:', l)]
flag = 0; total = 0; flagged_syms = []
for si in starts:
    sym = asm[si].split(':')[0]
    end = next(i for i in range(si + 1, len(asm)) if asm[i].startswith('.Lfunc_end'))
    body = asm[si:end]
    total += 1
    parents = {}          # header -> list of parent headers
    cur_loops = []        # loops of the current block
    loop_has_bar = defaultdict(bool); loop_div = defaultdict(bool)
    i = 0
    while i < len(body):
        l = body[i]
        m = re.match(r'^(?:\.L(BB\d+_\d+)|; %bb\.\d+):', l)
        if m:
            hm = re.search(r'Header=(BB\d+_\d+)', l)
            if 'This Loop Header' in l or 'This Inner Loop Header' in l:
                name = m.group(1)
                ps = []
                k = i - 1
                while k >= 0 and body[k].strip().startswith(';') and 'Parent Loop' in body[k]:
                    ps.append(re.search(r'Parent Loop (BB\d+_\d+)', body[k]).group(1)); k -= 1
                # parents may also be listed on following comment lines
                parents[name] = ps
                cur = [name] + ps
            elif hm:
                h = hm.group(1)
                cur = [h] + parents.get(h, [])
            else:
                cur = []
            cur_loops = cur
        t = l.strip()
        if t.startswith('s_barrier'):
            for h in cur_loops: loop_has_bar[h] = True
        if 's_andn2_b64 exec, exec' in t:
            for h in cur_loops[:1]: loop_div[h] = True
        i += 1
    for h in loop_div:
        if loop_has_bar[h]:
            flag += 1; flagged_syms.append(sym)
            if len(sys.argv) > 2: print('DIVERGENT LOOP WITH BARRIER', sym[:100], h)
print('kernels checked', total, 'flagged loops', flag, 'kernels', len(set(flagged_syms)))
sys.exit(1 if flag else 0)
