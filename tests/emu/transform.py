"""Source rewrite for the host emulation (test infrastructure only).

Kernel launches K<<<g, b, lds, s>>>(args) become emu_launch(...) calls whose
arguments are evaluated at the launch (as a graph node records them), and
the dynamic shared-memory declaration becomes a pointer to the emulated LDS.
"""
import re, sys
src = open(sys.argv[1]).read()
src = src.replace('extern __shared__ __attribute__((aligned(16))) double sm[];', 'double* sm = (double*)emu_dyn_lds;')

def split_top(s):
    out, depth, cur = [], 0, ''
    for ch in s:
        if ch in '([{<' and not (ch == '<' and False):
            depth += ch in '([{'
        if ch in ')]}':
            depth -= 1
        if ch == ',' and depth == 0:
            out.append(cur.strip()); cur = ''
        else:
            cur += ch
    if cur.strip():
        out.append(cur.strip())
    return out

res, i = '', 0
pat = re.compile(r'([A-Za-z_][A-Za-z0-9_:<>]*)<<<(.*?)>>>\(')
while True:
    m = pat.search(src, i)
    if not m:
        res += src[i:]; break
    res += src[i:m.start()]
    kern, cfg = m.group(1), split_top(m.group(2))
    j, depth = m.end(), 1
    while depth:
        if src[j] == '(':
            depth += 1
        elif src[j] == ')':
            depth -= 1
        j += 1
    args = split_top(src[m.end():j - 1])
    g, b = cfg[0], cfg[1]
    lds = cfg[2] if len(cfg) > 2 else '0'
    s = cfg[3] if len(cfg) > 3 else 'nullptr'
    binds = ''.join(f'auto _a{k} = ({a}); ' for k, a in enumerate(args))
    call = f'{kern}({", ".join(f"_a{k}" for k in range(len(args)))})'
    res += f'[&]{{ {binds}emu_launch(dim3({g}), dim3({b}), (size_t)({lds}), (hipStream_t)({s}), [=]() {{ {call}; }}); }}()'
    i = j
sys.stdout.write(res)
