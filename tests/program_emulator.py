"""CPU model of the lowered device program (tests only).

Interprets the JSON plan of ``qsv_plan_json`` the way the HIP kernels do:
tile index arithmetic (tile bases from the insert-zero masks, element
offsets from the tile-bit deposit), register subcube groups (subcube base
with zeros inserted at the group bits, element offsets), the Z-parity tables
and the per-slot inner products.  It shares no code with the oracle; it lets
the CPU suite check planning and lowering against the oracle without a GPU.
The streaming single-gate passes are modelled by their index sets.
"""
import numpy as np

OP_APPLY1, OP_APPLY2, OP_APPLYK, OP_DIAG, OP_ZPHASE, OP_DOT1, OP_DOT2, OP_DOTK, OP_DOTDIAG, OP_DOTZSUM, OP_GROUP, \
    OP_LAYER1, OP_ZPHDOT = range(1, 14)
MC_DENSE, MC_DIAG, MC_ANTI, MC_MID, MC_REAL, MC_RIRI, MC_PX, MC_PY, MC_RIRI_D, MC_RIRI_O, MC_REAL_D, MC_REAL_O = range(12)


def _coef(prog, off, cnt):
    c = prog["_coef"]
    return c[off:off + cnt]


def expand(k, masks):
    r = k & masks[0]
    for i in range(1, len(masks)):
        r |= (k << i) & masks[i]
    return r


def popc(x):
    return bin(x).count("1")


def parity_bits(x, z):
    p = 0
    for j, zm in enumerate(z):
        p |= (popc(x & zm) & 1) << j
    return p


def run_program(prog, phi, lam=None, slots=None):
    """Apply every pass of the program to phi (and lam); inner products are
    added to slots[slot_base + slot]."""
    prog["_coef"] = np.array(prog["coef"], dtype=float).view(np.complex128)
    for st in prog["steps"]:
        if st["type"] == "tile":
            _tile(prog, st, phi, lam, slots)
        else:
            _stream(prog, st, phi)


def _dense(prog, st, psi):
    """The LDS-staged dense kernel, index by index: 256 threads load the tile
    (tile-local index tid + r * 256 -> global offset and compact LDS index by
    bit deposits), wave w computes rows [w R, (w+1) R) of the 64 tuples (lane
    = tuple) from the padded LDS layout, and the outputs go back the same way."""
    k = st["k"]
    D = 1 << k
    NT = st["nthr"]
    NW = NT // 64
    LB = NT.bit_length() - 1
    RW = D // NW
    RL = (64 << k) // NT
    # the kernel's layout: (wave, column j, row q of the wave's RW rows)
    Mt = _coef(prog, st["coff"], D * D).reshape(NW, D, RW)
    M = np.concatenate([Mt[w].T for w in range(NW)], axis=0)
    sb, cb = st["sb"], st["cb"]
    lds_size = (64 << k) * 65 // 64
    for tile in range(st["n_tiles"]):
        base = expand(tile, st["outer"]) | st["setmask"]
        lds = np.full(lds_size, np.nan + 0j)
        slots = []
        for tid in range(NT):
            goff = sum(1 << sb[i] for i in range(LB) if (tid >> i) & 1)
            coff = sum(1 << cb[i] for i in range(LB) if (tid >> i) & 1)
            for r in range(RL):
                g = base | goff | st["goff_hi"][r]
                c = coff | st["coff_hi"][r]
                assert c + (c >> 6) < lds_size
                lds[c + (c >> 6)] = psi[g]
                slots.append((g, c))
        assert len({g for g, _ in slots}) == 64 << k and len({c for _, c in slots}) == 64 << k
        out = lds.copy()
        for wave in range(NW):
            for lane in range(64):
                x = np.array([lds[(j << 6) + lane + j] for j in range(D)])
                for q in range(RW):
                    row = wave * RW + q
                    out[(row << 6) + lane + row] = M[row] @ x
        for g, c in slots:
            psi[g] = out[c + (c >> 6)]


def _stream(prog, st, psi):
    if st["type"] == "dense":
        _dense(prog, st, psi)
        return
    ex = st["ex"]
    idx = np.array([expand(k, ex) | st["setmask"] for k in range(st["n_items"])], dtype=np.int64)
    m2 = np.array(st["m2"], dtype=float).view(np.complex128)
    m4 = np.array(st["m4"], dtype=float).view(np.complex128)
    if st["type"] == "diag1":
        psi[idx] *= st["dre"] + 1j * st["dim"]
    elif st["type"] == "gate1":
        i0, i1 = idx, idx | st["tbit"]
        a0, a1 = psi[i0].copy(), psi[i1].copy()
        psi[i0] = m2[0] * a0 + m2[1] * a1
        psi[i1] = m2[2] * a0 + m2[3] * a1
    elif st["type"] == "gate2":
        b0, b1 = st["b0"], st["b1"]
        ids = [idx, idx | b1, idx | b0, idx | b0 | b1]
        a = [psi[i].copy() for i in ids]
        M = m4.reshape(4, 4)
        for r in range(4):
            psi[ids[r]] = sum(M[r, j] * a[j] for j in range(4))
    elif st["type"] == "gatek_low":
        # chunks of 64 amplitudes (index bits above 5 from ex / setmask); one
        # output per lane: its row from its target bits, inputs from its tuple
        k = st["k"]
        D = 1 << k
        M = _coef(prog, st["coff"], D * D).reshape(D, D)
        tb = st["tb"][:k]
        assert max(tb) < 6
        tmask = sum(1 << t for t in tb)
        for c in range(st["n_items"]):
            base = (expand(c, ex) | st["setmask"]) << 6
            chunk = psi[base:base + 64].copy()
            for lane in range(64):
                if (lane & st["lcm"]) != st["lcv"]:
                    continue
                row = 0
                for t in tb:
                    row = (row << 1) | ((lane >> t) & 1)
                t0 = lane & ~tmask
                acc = 0j
                for j in range(D):
                    o = t0
                    for i in range(k):
                        if (j >> (k - 1 - i)) & 1:
                            o |= 1 << tb[i]
                    acc += M[row, j] * chunk[o]
                psi[base + lane] = acc
    else:
        k = st["k"]
        D = 1 << k
        M = _coef(prog, st["coff"], D * D).reshape(D, D)
        offs = []
        for j in range(D):
            o = 0
            for i in range(k):
                if (j >> (k - 1 - i)) & 1:
                    o |= 1 << st["tb"][i]
            offs.append(o)
        a = np.stack([psi[idx | o] for o in offs])
        out = M @ a
        for j, o in enumerate(offs):
            psi[idx | o] = out[j]


def _tile(prog, st, phi, lam, slots):
    b, nthr, R = st["b"], st["nthr"], st["R"]
    sb = st["sb"]
    tsz = 1 << b
    # element t = tid + r * nthr -> deposit into the tile bits
    dep = np.zeros(tsz, dtype=np.int64)
    for t in range(tsz):
        o = 0
        for j in range(b):
            if (t >> j) & 1:
                o |= 1 << sb[j]
        dep[t] = o
    tops = prog["tops"][st["op0"]:st["op0"] + st["nops"]]
    two = lam is not None
    for T in range(st["n_tiles"]):
        base = expand(T, st["outer"])
        g = base | dep
        tp = phi[g].copy()
        tl = lam[g].copy() if two else None
        i = 0
        while i < len(tops):
            op = tops[i]
            if op["kind"] == OP_GROUP:
                _group(prog, st, op, tops[i + 1:i + 1 + op["m"]], tp, tl, base, slots, T)
                i += 1 + op["m"]
                continue
            _standalone(prog, st, op, tp, tl, base, dep, slots, T)
            i += 1
        # factored layers leave the tile divided by the pass's scale
        sc = st.get("out_scale", 1.0)
        phi[g] = tp * sc
        if two:
            lam[g] = tl * sc


def _tile_parity(w, off, n_outer, T):
    """Parity bits of the tile base from the per-outer-bit columns (the
    kernel's form: XOR of the columns of the tile number's set bits)."""
    pb = 0
    for k in range(n_outer):
        if (T >> k) & 1:
            pb ^= w[off + k]
    return pb


def _group(prog, st, g, subs, tp, tl, base, slots, T):
    b = st["b"]
    GB = g["k"]
    Q = g["tb"][:GB]
    E = 1 << GB
    nsub = (1 << b) >> GB
    w = prog["words"]
    eo = np.array([sum(((e >> i) & 1) << Q[i] for i in range(GB)) for e in range(E)], dtype=np.int64)
    geo = np.array(w[g["woff"]:g["woff"] + E], dtype=np.int64)
    gpos = w[g["woff"] + E:g["woff"] + E + b - GB]
    sc = np.arange(nsub, dtype=np.int64)
    tc = sc.copy()
    for q in Q:
        tc = ((tc >> q) << (q + 1)) | (tc & ((1 << q) - 1))
    gc = np.full(nsub, base, dtype=np.int64)
    for j, p in enumerate(gpos):
        gc |= ((sc >> j) & 1) << p
    idx = tc[:, None] | eo[None, :]            # [subcube, element] -> tile index
    gi = gc[:, None] | geo[None, :]             # global index
    a = tp[idx]
    l = tl[idx] if tl is not None else None
    for s in subs:
        kind = s["kind"]
        local = kind in (OP_APPLY1, OP_APPLY2, OP_DOT1, OP_DOT2)
        if local and (base & s["gcmask"]) != s["gcval"]:
            continue
        ok = ((idx & s["lcmask"]) == s["lcval"])
        if kind in (OP_APPLY1, OP_DOT1):
            P = s["tb"][0]
            m = _coef(prog, s["coff"], 4)
            for e0 in range(E):
                if e0 & (1 << P):
                    continue
                e1 = e0 | (1 << P)
                sel = ok[:, e0]
                if kind == OP_APPLY1:
                    for x in ([a, l] if l is not None else [a]):
                        x0, x1 = x[sel, e0].copy(), x[sel, e1].copy()
                        if s["cls"] == MC_ANTI:
                            x[sel, e0], x[sel, e1] = m[1] * x1, m[2] * x0
                        else:
                            x[sel, e0], x[sel, e1] = m[0] * x0 + m[1] * x1, m[2] * x0 + m[3] * x1
                else:
                    p0, p1 = a[sel, e0], a[sel, e1]
                    v = (np.conj(l[sel, e0]) * (m[0] * p0 + m[1] * p1) + np.conj(l[sel, e1]) * (m[2] * p0 + m[3] * p1))
                    slots[st["slot_base"] + s["slot"]] += v.imag.sum()
        elif kind in (OP_APPLY2, OP_DOT2):
            P0, P1 = s["tb"][0], s["tb"][1]
            m = _coef(prog, s["coff"], 16).reshape(4, 4)
            for e in range(E):
                if e & ((1 << P0) | (1 << P1)):
                    continue
                ids = [e, e | (1 << P1), e | (1 << P0), e | (1 << P0) | (1 << P1)]
                sel = ok[:, e]
                if kind == OP_APPLY2:
                    for x in ([a, l] if l is not None else [a]):
                        y = [x[sel, i].copy() for i in ids]
                        if s["cls"] == MC_MID:
                            x[sel, ids[1]] = m[1, 1] * y[1] + m[1, 2] * y[2]
                            x[sel, ids[2]] = m[2, 1] * y[1] + m[2, 2] * y[2]
                        else:
                            for r in range(4):
                                x[sel, ids[r]] = sum(m[r, j] * y[j] for j in range(4))
                else:
                    y = [a[sel, i] for i in ids]
                    v = sum(np.conj(l[sel, ids[r]]) * sum(m[r, j] * y[j] for j in range(4)) for r in range(4))
                    slots[st["slot_base"] + s["slot"]] += v.imag.sum()
        elif kind in (OP_DIAG, OP_DOTDIAG):
            assert g["aux"] == 1, "the kernel computes global indices only for groups flagged aux = 1"
            k = s["k"]
            d = _coef(prog, s["coff"], 1 << k)
            j = np.zeros_like(gi)
            for i in range(k):
                j = (j << 1) | ((gi >> s["tb"][i]) & 1)
            on = (gi & s["gcmask"]) == s["gcval"]
            dd = np.where(on, d[j], 1.0)
            if kind == OP_DIAG:
                a *= dd
                if l is not None:
                    l *= dd
            else:
                v = np.where(on, np.conj(l) * d[j] * a, 0)
                slots[st["slot_base"] + s["slot"]] += v.imag.sum()
        elif kind in (OP_ZPHASE, OP_DOTZSUM, OP_ZPHDOT):
            mz = s["m"]
            z = w[s["woff"]:s["woff"] + mz]
            pb = _tile_parity(w, s["woff"] + mz + nsub + E, st["n_outer"], T)
            assert pb == parity_bits(base, z)
            pcs = np.array(w[s["woff"] + mz:s["woff"] + mz + nsub], dtype=np.int64)
            pes = np.array(w[s["woff"] + mz + nsub:s["woff"] + mz + nsub + E], dtype=np.int64)
            cnt = np.vectorize(popc)(pb ^ pcs[:, None] ^ pes[None, :])
            if kind in (OP_DOTZSUM, OP_ZPHDOT):
                v = (mz - 2 * cnt) * (np.conj(l) * a).imag
                slots[st["slot_base"] + s["slot"]] += v.sum()
            if kind in (OP_ZPHASE, OP_ZPHDOT):
                if kind == OP_ZPHDOT:  # the kernel reads the pass's LDS copy of the tables at lcval
                    assert s["coff"] == st["zt_off"] + s["lcval"] and s["lcval"] + mz + 1 <= st["zt_n"]
                else:
                    assert s["coff"] == st["zt_off"] + s["aux"] and s["aux"] + mz + 1 <= st["zt_n"]
                d = _coef(prog, s["coff"], mz + 1)[cnt]
                a *= d
                if l is not None:
                    l *= d
        elif kind == OP_LAYER1:
            # per position P ascending: optional inner product, then the 2x2
            gcode = s["lcval"]  # 0 none, 1 X, 2 Y, 3 dense, 4 real diagonal
            assert gcode in (0, 1, 2, 3, 4) and (gcode == 0) == (s["lcmask"] == 0)
            nc = 8 if gcode in (3, 4) else 4
            cf = _coef(prog, s["coff"], nc * GB)
            for P in range(GB):
                mp = cf[P * nc:(P + 1) * nc]
                M = mp[4:8] if gcode in (3, 4) else mp[:4]
                if s["cls"] == MC_REAL:
                    assert np.all(M.imag == 0)
                elif s["cls"] == MC_DIAG:
                    assert M[1] == 0 and M[2] == 0
                elif s["cls"] in (MC_RIRI_D, MC_REAL_D):  # factored: unit diagonal
                    assert M[0] == 1 and M[3] == 1
                elif s["cls"] == MC_RIRI_O:
                    assert M[1] == 1j and M[2] == 1j
                elif s["cls"] == MC_REAL_O:
                    assert M[1] == -1 and M[2] == 1
                elif s["cls"] == MC_RIRI:
                    assert M[0].imag == 0 and M[3].imag == 0 and M[1].real == 0 and M[2].real == 0
                pairs = [(e0, e0 | (1 << P)) for e0 in range(E) if not e0 & (1 << P)]
                if (s["lcmask"] >> P) & 1:
                    assert l is not None
                    G = {1: np.array([0, 1, 1, 0], dtype=complex),
                         2: np.array([0, -1j, 1j, 0])}.get(gcode, mp[:4])
                    if gcode == 4:
                        assert G[1] == 0 and G[2] == 0 and G[0].imag == 0 and G[3].imag == 0
                    v = 0.0
                    for e0, e1 in pairs:
                        p0, p1 = a[:, e0], a[:, e1]
                        v += (np.conj(l[:, e0]) * (G[0] * p0 + G[1] * p1) +
                              np.conj(l[:, e1]) * (G[2] * p0 + G[3] * p1)).imag.sum()
                    slots[st["slot_base"] + s["tb"][P]] += v
                if not (s["m"] >> P) & 1:
                    assert np.all(M == np.array([1, 0, 0, 1]))  # no gate here: the table holds I
                    continue
                for x in ([a, l] if l is not None else [a]):
                    for e0, e1 in pairs:
                        x0, x1 = x[:, e0].copy(), x[:, e1].copy()
                        x[:, e0], x[:, e1] = M[0] * x0 + M[1] * x1, M[2] * x0 + M[3] * x1
        else:
            raise AssertionError(f"op kind {kind} inside a group")
    tp[idx] = a
    if tl is not None:
        tl[idx] = l


def _standalone(prog, st, op, tp, tl, base, dep, slots, T):
    kind = op["kind"]
    b, nthr, R = st["b"], st["nthr"], st["R"]
    tsz = 1 << b
    t = np.arange(tsz, dtype=np.int64)
    gi = base | dep
    if kind in (OP_APPLY1, OP_APPLY2, OP_APPLYK, OP_DOT1, OP_DOT2, OP_DOTK) and (base & op["gcmask"]) != op["gcval"]:
        return
    if kind in (OP_APPLY1, OP_APPLY2, OP_APPLYK, OP_DOT1, OP_DOT2, OP_DOTK):
        k = op["k"]
        D = 1 << k
        tmask = sum(1 << op["tb"][i] for i in range(k))
        G = _coef(prog, op["coff"], D * D).reshape(D, D)
        gb = t[(t & tmask) == 0]
        gb = gb[(gb & op["lcmask"]) == op["lcval"]]
        offs = [sum(((j >> (k - 1 - i)) & 1) << op["tb"][i] for i in range(k)) for j in range(D)]
        ids = np.stack([gb | o for o in offs])
        if kind in (OP_APPLY1, OP_APPLY2, OP_APPLYK):
            for x in ([tp, tl] if tl is not None else [tp]):
                x[ids] = G @ x[ids]
        else:
            v = np.sum(np.conj(tl[ids]) * (G @ tp[ids]))
            slots[st["slot_base"] + op["slot"]] += v.imag
    elif kind in (OP_DIAG, OP_DOTDIAG):
        k = op["k"]
        d = _coef(prog, op["coff"], 1 << k)
        j = np.zeros_like(gi)
        for i in range(k):
            j = (j << 1) | ((gi >> op["tb"][i]) & 1)
        on = (gi & op["gcmask"]) == op["gcval"]
        if kind == OP_DIAG:
            dd = np.where(on, d[j], 1.0)
            tp *= dd
            if tl is not None:
                tl *= dd
        else:
            slots[st["slot_base"] + op["slot"]] += np.where(on, np.conj(tl) * d[j] * tp, 0).imag.sum()
    else:  # ZPHASE / DOTZSUM with per-thread and per-r parity tables
        w = prog["words"]
        mz = op["m"]
        z = w[op["woff"]:op["woff"] + mz]
        pb = _tile_parity(w, op["woff"] + mz + nthr + R, st["n_outer"], T)
        assert pb == parity_bits(base, z)
        plo = w[op["woff"] + mz:op["woff"] + mz + nthr]
        phi_r = w[op["woff"] + mz + nthr:op["woff"] + mz + nthr + R]
        cnt = np.array([popc(pb ^ plo[int(x) % nthr] ^ phi_r[int(x) // nthr]) for x in t])
        if kind == OP_ZPHASE:
            d = _coef(prog, op["coff"], mz + 1)[cnt]
            tp *= d
            if tl is not None:
                tl *= d
        else:
            slots[st["slot_base"] + op["slot"]] += ((mz - 2 * cnt) * (np.conj(tl) * tp).imag).sum()


def emulate_apply(n, ops, params, psi0, **opts):
    from paper_2403_02512_amd import qsv
    prog = qsv.plan_json(n, ops, params, **opts)
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    run_program(prog, psi)
    return psi


def emulate_adjoint(n, ops, params, psi, lam, **opts):
    """One reverse sweep from phi = psi, lambda = lam; returns the gradient."""
    from paper_2403_02512_amd import qsv
    prog = qsv.plan_json(n, ops, params, adjoint=True, **opts)
    phi = np.array(psi, dtype=np.complex128, copy=True)
    lm = np.array(lam, dtype=np.complex128, copy=True)
    slots = np.zeros(len(prog["slot_param"]))
    run_program(prog, phi, lm, slots)
    grad = np.zeros(len(params))
    for s, (p, c) in enumerate(prog["slot_param"]):
        grad[p] += c * slots[s]
    return grad, phi
