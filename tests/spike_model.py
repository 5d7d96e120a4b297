"""Dense NumPy statement of the SPIKE algebra used by the solver (test aid).

Not the oracle: it restates, on tiny dense matrices, the decomposition the
GPU path implements (leaf spike tips V_i = A_i^{-1} B_i, W_i = A_i^{-1} C_i;
pairwise merges of adjacent nodes through the interface system
E_J = [[I, Vb_L], [Wt_R, I]]; node tips; bottom-up then top-down reduced
solve; retrieval; and the transpose solve as the adjoint of those passes), so
tests can check the intermediate identities of the paper's DS factorisation
and recursive reduced system against dense linear algebra.
"""
import numpy as np


def merge_tree(p):
    """Pair adjacent nodes left to right per level; an odd last node carries
    up.  Returns merges as dicts (interface, left id, right id, a, b, level)."""
    cur = [(i, i, i) for i in range(p)]
    merges, level = [], 0
    while len(cur) > 1:
        level += 1
        nxt = []
        for i in range(0, len(cur), 2):
            if i + 1 < len(cur):
                (a, m, lid), (_, b, rid) = cur[i], cur[i + 1]
                merges.append(dict(mif=m, left=lid, right=rid, a=a, b=b, level=level))
                nxt.append((a, b, p + m))
            else:
                nxt.append(cur[i])
        cur = nxt
    return merges, level


def tree_from_spans(p, spans):
    """Merge dicts from (level, a, m, b) tuples in launch order: the left child
    spans leaves a..m and the right m+1..b.  A child must be a leaf or a node
    an earlier merge formed (else KeyError)."""
    owner = {(i, i): i for i in range(p)}
    merges = []
    for level, a, m, b in spans:
        merges.append(dict(mif=m, left=owner[(a, m)], right=owner[(m + 1, b)], a=a, b=b, level=level))
        owner[(a, b)] = p + m
    return merges, max((s[0] for s in spans), default=0)


class Model:
    def __init__(self, A, sizes, kl, ku, tree=None):
        """tree: (merges, levels) as merge_tree returns; the balanced tree by
        default."""
        self.A, self.kl, self.ku = A, kl, ku
        self.sizes = list(sizes)
        self.p = p = len(sizes)
        self.starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)
        self.merges, self.levels = tree if tree is not None else merge_tree(p)
        self.tips = {}
        for i in range(p):
            s, m = self.starts[i], self.sizes[i]
            Ai = A[s:s + m, s:s + m]
            t = {}
            if i < p - 1:
                V = np.linalg.solve(Ai, A[s:s + m, s + m:s + m + ku])
                t["Vt"], t["Vb"] = V[:ku], V[m - kl:]
            if i > 0:
                W = np.linalg.solve(Ai, A[s:s + m, s - kl:s])
                t["Wt"], t["Wb"] = W[:ku], W[m - kl:]
            self.tips[i] = t
        self.fac = {}
        for J in self.merges:
            L, R = self.tips[J["left"]], self.tips[J["right"]]
            P, Q = L["Vb"], R["Wt"]
            S = np.eye(ku) - Q @ P
            f = dict(S=S, P=P, Q=Q, alpha=np.zeros((kl, ku)), beta=np.zeros((ku, ku)),
                     gamma=np.zeros((kl, kl)), delta=np.zeros((ku, kl)))
            nv, nw = J["b"] < p - 1, J["a"] > 0
            if nv:
                f["beta"] = np.linalg.solve(S, R["Vt"])
                f["alpha"] = -P @ f["beta"]
            if nw:
                f["delta"] = -np.linalg.solve(S, Q @ L["Wb"])
                f["gamma"] = L["Wb"] - P @ f["delta"]
            t = {}
            if nv and nw:
                t["Vt"] = -L["Vt"] @ f["beta"]
                t["Wb"] = -R["Wb"] @ f["gamma"]
            if nv:
                t["Vb"] = R["Vb"] - R["Wb"] @ f["alpha"]
            if nw:
                t["Wt"] = L["Wt"] - L["Vt"] @ f["delta"]
            self.tips[p + J["mif"]] = t
            self.fac[J["mif"]] = f

    def block(self, i):
        s, m = self.starts[i], self.sizes[i]
        return self.A[s:s + m, s:s + m]

    # --------------------------------------------------------------- A X = F
    def solve(self, F):
        A, kl, ku, p = self.A, self.kl, self.ku, self.p
        F = np.atleast_2d(F.T).T if F.ndim == 1 else F
        Y, val = {}, {}
        for i in range(p):
            s, m = self.starts[i], self.sizes[i]
            Y[i] = np.linalg.solve(self.block(i), F[s:s + m])
            val[i] = dict(top=Y[i][:ku], bot=Y[i][m - kl:])
        st = {}
        for J in self.merges:                      # bottom-up
            f, L, R = self.fac[J["mif"]], val[J["left"]], val[J["right"]]
            t = np.linalg.solve(f["S"], R["top"] - f["Q"] @ L["bot"])
            s_ = L["bot"] - f["P"] @ t
            st[J["mif"]] = (s_, t)
            v = {}
            if J["a"] > 0:
                v["top"] = L["top"] - self.tips[J["left"]]["Vt"] @ t
            if J["b"] < p - 1:
                v["bot"] = R["bot"] - self.tips[J["right"]]["Wb"] @ s_
            val[p + J["mif"]] = v
        x = {}
        for J in reversed(self.merges):            # top-down
            f = self.fac[J["mif"]]
            xb, xt = st[J["mif"]]
            xb, xt = xb.copy(), xt.copy()
            if J["b"] < p - 1:
                xr = x[J["b"]][1]
                xb -= f["alpha"] @ xr
                xt -= f["beta"] @ xr
            if J["a"] > 0:
                xl = x[J["a"] - 1][0]
                xb -= f["gamma"] @ xl
                xt -= f["delta"] @ xl
            x[J["mif"]] = (xb, xt)
        X = np.zeros_like(F)
        for i in range(p):                         # retrieval
            s, m = self.starts[i], self.sizes[i]
            c = np.zeros((m, F.shape[1]))
            if i < p - 1:
                c += A[s:s + m, s + m:s + m + ku] @ x[i][1]
            if i > 0:
                c += A[s:s + m, s - kl:s] @ x[i - 1][0]
            X[s:s + m] = Y[i] - np.linalg.solve(self.block(i), c)
        self.last_x = x
        return X

    # --------------------------------------------------------------- A^T X = F
    def solve_t(self, F):
        A, kl, ku, p = self.A, self.kl, self.ku, self.p
        Z = {}
        for i in range(p):
            s, m = self.starts[i], self.sizes[i]
            g = F[s:s + m].copy()
            if i > 0:
                g[:ku] = 0
            if i < p - 1:
                g[m - kl:] = 0
            Z[i] = np.linalg.solve(self.block(i).T, g)
        xbar = {}
        for mi in range(p - 1):
            s, m = self.starts[mi], self.sizes[mi]
            s1 = self.starts[mi + 1]
            Chat = A[s1:s1 + kl, s1 - kl:s1]
            Bhat = A[s1 - ku:s1, s1:s1 + ku]
            gb = F[s + m - kl:s + m] - Chat.T @ Z[mi + 1][:kl]
            gt = F[s1:s1 + ku] - Bhat.T @ Z[mi][self.sizes[mi] - ku:]
            xbar[mi] = [gb, gt]
        crl, sbar = {}, {}
        for d, J in enumerate(self.merges):        # adjoint of top-down, bottom-up
            f = self.fac[J["mif"]]
            xb, xt = xbar[J["mif"]]
            sbar[J["mif"]] = [xb.copy(), xt.copy()]
            if J["b"] < p - 1:
                xbar[J["b"]][1] = xbar[J["b"]][1] - (f["alpha"].T @ xb + f["beta"].T @ xt)
            if J["a"] > 0:
                xbar[J["a"] - 1][0] = xbar[J["a"] - 1][0] - (f["gamma"].T @ xb + f["delta"].T @ xt)
        ybar = {}
        for J in reversed(self.merges):            # adjoint of bottom-up, top-down
            f = self.fac[J["mif"]]
            sb, tb = sbar[J["mif"]]
            yj = ybar.get(p + J["mif"], {})
            if J["a"] > 0:
                tb = tb - self.tips[J["left"]]["Vt"].T @ yj["top"]
            if J["b"] < p - 1:
                sb = sb - self.tips[J["right"]]["Wb"].T @ yj["bot"]
            v = np.linalg.solve(f["S"].T, tb - f["P"].T @ sb)
            u = sb - f["Q"].T @ v
            yl = ybar.setdefault(J["left"], {})
            yr = ybar.setdefault(J["right"], {})
            yl["bot"], yr["top"] = u, v
            if J["a"] > 0:
                yl["top"] = yj["top"]
            if J["b"] < p - 1:
                yr["bot"] = yj["bot"]
        X = np.zeros_like(F)
        for i in range(p):
            s, m = self.starts[i], self.sizes[i]
            g = F[s:s + m].copy()
            if p > 1:
                if i > 0:
                    g[:ku] = ybar[i]["top"]
                if i < p - 1:
                    g[m - kl:] = ybar[i]["bot"]
            X[s:s + m] = np.linalg.solve(self.block(i).T, g)
        return X
