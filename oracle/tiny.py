"""Pure-Python, set-based transcription of Algorithm 1 for tiny domains.

TEST INFRASTRUCTURE ONLY (an independent second oracle; it shares nothing with
the C oracle or the HIP path).  Written from the paper's definitions in their
own terms, with Python sets:

* Omega_h = lattice points of the image; D^(k)_h, B_h as sets of (x, y);
* the active boundary (Notation): points of D^(k)_h with a point of
  Omega_h \\ (D^(k)_h u B_h) among their eight neighbours (the inner-boundary
  condition then holds automatically);
* the continuous sets D^(k), B (Notation): every point within L-infinity
  distance < 1 of a pixel of D^(k)_h resp. B_h; a ghost point p is usable iff
  p lies in the closed image rectangle Omega and in neither set;
* u is extended to usable points by the bilinear basis (eqn:bilinearDef):
  u(p) = sum over lattice y of max(0, 1 - |p_x - y_x|) max(0, 1 - |p_y - y_y|) u(y);
* the rotated ball R(B_eps(x)) with R taking (0,1) to g/|g| (Sec. 3.1), the
  lattice ball when g = 0 or in coherence-transport mode;
* weights eqn:weight, confidence eqn:confidence, ready eqn:ready (onion order
  when c < 0: every active pixel with a usable point is filled); with c2 >= 0
  the data term of eqn:ready2, D(x) = |g(x)| > c2, gates ready until a shell
  fills nothing, after which eqn:ready alone decides (that shell is taken
  again);
* the shell update of Algorithm 1 with the state of shell k frozen while
  shell k is computed.

Distances to lattice points are compared as exact inequalities on the offset
from x (d - 1 < o < d + 1), never as rounded absolute positions.  The
quotient of Algorithm 1 is evaluated with every weight divided by the largest
usable one (same value, no underflow).
"""

from __future__ import annotations

import math


def ball(eps: float):
    R = int(math.floor(eps))
    out = []
    for m in range(-R, R + 1):
        for n in range(-R, R + 1):
            if (n, m) != (0, 0) and n * n + m * m <= eps * eps:
                out.append((n, m))
    return out


def rotated_offset(gx: float, gy: float, n: int, m: int, ghost: bool):
    """R(n, m) with R the rotation taking (0, 1) to g/|g|; (n, m) if not rotating."""
    if ghost and (gx != 0.0 or gy != 0.0):
        L = math.sqrt(gx * gx + gy * gy)
        c = gx / L
        s = gy / L
        # R(1,0) = (s, -c), R(0,1) = (c, s); evaluated as n*s + m*c and m*s - n*c
        return (n * s + m * c, m * s - n * c)
    return (float(n), float(m))


def fill(img, label, guide, eps=3.0, mu=50.0, c=-1.0, ghost=True, max_shells=0, c2=-1.0):
    """img: H x W x C nested lists or array; label: H x W; guide: H x W x 2.
    Returns (u as H x W x C list of floats, shell map as H x W list, K)."""
    H = len(label)
    W = len(label[0])
    C = len(img[0][0])
    u = {(x, y): [float(img[y][x][ch]) for ch in range(C)] for y in range(H) for x in range(W)}
    Omega = {(x, y) for y in range(H) for x in range(W)}
    Dk = {(x, y) for (x, y) in Omega if label[y][x] == 1}
    Bh = {(x, y) for (x, y) in Omega if label[y][x] == 2}
    shell = {}
    for (x, y) in Omega:
        shell[(x, y)] = -1 if label[y][x] == 0 else (-2 if label[y][x] == 2 else -3)
    a = mu * mu / (2.0 * eps * eps)
    offs = ball(eps)
    nbr8 = [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dx, dy) != (0, 0)]
    K = 0
    k = 0
    data_phase = c2 >= 0.0
    while True:
        if not Dk:
            break
        if max_shells and k >= max_shells:
            break
        blocked = Dk | Bh  # D^(k)_h u B_h
        readable_h = Omega - blocked
        active = [p for p in Dk if any((p[0] + dx, p[1] + dy) in readable_h for dx, dy in nbr8)]
        new_vals = {}
        for (x, y) in active:
            gx, gy = float(guide[y][x][0]), float(guide[y][x][1])
            if data_phase and not (math.sqrt(gx * gx + gy * gy) > c2):
                continue
            pts = []
            for (n, m) in offs:
                ox, oy = rotated_offset(gx, gy, n, m, ghost)
                # in the closed rectangle Omega: 0 <= x + ox <= W - 1, same for y
                inside = (-x <= ox <= (W - 1) - x) and (-y <= oy <= (H - 1) - y)
                usable = inside
                if usable:
                    for (bx, by) in blocked:
                        ddx, ddy = bx - x, by - y
                        if ddx - 1 < ox < ddx + 1 and ddy - 1 < oy < ddy + 1:
                            usable = False
                            break
                t = -gy * ox + gx * oy
                logw = -a * t * t - math.log(math.hypot(ox, oy))
                pts.append((ox, oy, usable, logw))
            use = [p for p in pts if p[2]]
            if not use:
                continue
            if c >= 0.0:
                top_all = max(p[3] for p in pts)
                den = sum(math.exp(p[3] - top_all) for p in pts)
                num = sum(math.exp(p[3] - top_all) for p in use)
                if not (num / den > c):
                    continue
            top = max(p[3] for p in use)
            S = 0.0
            acc = [0.0] * C
            for (ox, oy, _, logw) in use:
                w = math.exp(logw - top)
                S += w
                val = [0.0] * C
                R = int(math.floor(eps)) + 2
                for ddy in range(-R, R + 1):
                    ly = 1.0 - abs(oy - ddy)
                    if ly <= 0:
                        continue
                    for ddx in range(-R, R + 1):
                        lx = 1.0 - abs(ox - ddx)
                        if lx <= 0:
                            continue
                        q = (x + ddx, y + ddy)
                        for ch in range(C):
                            val[ch] += lx * ly * u[q][ch]
                for ch in range(C):
                    acc[ch] += w * val[ch]
            new_vals[(x, y)] = [acc[ch] / S for ch in range(C)]
        if not new_vals:
            if data_phase:  # the data term holds everything back: eqn:ready from here on
                data_phase = False
                continue
            break
        for p, v in new_vals.items():
            u[p] = v
            shell[p] = k
        Dk = Dk - set(new_vals)
        K = k + 1
        k += 1
    out_u = [[u[(x, y)] for x in range(W)] for y in range(H)]
    out_s = [[shell[(x, y)] for x in range(W)] for y in range(H)]
    return out_u, out_s, K
