"""Velocity sets of the oracle.

D2Q9: directions and weights as printed in Sec. III (the e and w arrays):
opposite directions sit next to each other (1<->2, 3<->4, 5<->6, 7<->8).

D3Q19: the paper only says the 3-D extension is the standard route (Sec. III,
after the D2Q9 weights).  We use the textbook D3Q19: rest weight 1/3, six face
neighbours 1/18, twelve edge neighbours 1/36, again with opposite pairs next to
each other.  Both sets have c_s^2 = 1/3 and delta t = 1.

Vectors are stored with three components (x, y, z); D2Q9 has e_z = 0 and the
oracle's arrays then carry a z axis of length one.
"""
import numpy as np

CS2 = 1.0 / 3.0


class Lattice:
    def __init__(self, name, e, w):
        self.name = name
        self.e = np.asarray(e, dtype=np.int64)          # [Q, 3]
        self.w = np.asarray(w, dtype=np.float64)        # [Q]
        self.Q = len(self.w)
        self.dim = 2 if name == "D2Q9" else 3
        opp = []
        for k in range(self.Q):
            match = [j for j in range(self.Q) if np.all(self.e[j] == -self.e[k])]
            assert len(match) == 1
            opp.append(match[0])
        self.opp = np.asarray(opp, dtype=np.int64)

    def __repr__(self):
        return f"Lattice({self.name})"


D2Q9 = Lattice(
    "D2Q9",
    e=[(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
       (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)],
    w=[4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
)

D3Q19 = Lattice(
    "D3Q19",
    e=[(0, 0, 0),
       (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
       (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
       (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
       (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)],
    w=[1 / 3] + [1 / 18] * 6 + [1 / 36] * 12,
)


def by_name(name):
    return {"D2Q9": D2Q9, "D3Q19": D3Q19}[name]
