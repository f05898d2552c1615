"""Local expectation values from the sandwich (Sec. 2, fig. Sandwich).

Test infrastructure only (see the package docstring).

After the boundaries from the top and from the bottom are known, the row in
the centre (or any row r) is contracted between T_{r-1} and B_{r+1}: a chain
of left and right environments over the columns.  Operators are inserted on
the ket layer, <O> = <psi|O|psi> / <psi|psi>, both numerator and denominator
taken from the same sandwich (a reading: the paper does not say how the ratio
is formed).  Vertical bonds couple two rows and are read from the two-row
sandwich between T_{r-1} and B_{r+2} (also a reading).

Index letters: o bottom-boundary bond, a/e top-boundary bond (left/right),
l/m left ket/bra legs, u/v up legs, r/s right legs, d/g down legs,
p/q physical; a trailing digit marks the second row.
"""
import numpy as np

from .spin import BOND_TERMS, SZ

EIN = dict(optimize=True)


def apply_op(O, A):
    """Operator on the physical leg of the ket tensor: sum_q O[p,q] A[q,...]."""
    return np.einsum("pq,qlurd->plurd", O, A, **EIN)


def row_step(L, T, Ak, Ab, B):
    """L'[o',r,s,e] = sum L[o,l,m,a] T[a,u,v,e] Ak[p,l,u,r,d] Ab[p,m,v,s,g] B[o,d,g,o']."""
    Y = np.einsum("olma,auve->olmuve", L, T, **EIN)
    Y = np.einsum("olmuve,plurd->omveprd", Y, Ak, **EIN)
    Y = np.einsum("omveprd,pmvsg->oerdsg", Y, Ab, **EIN)
    return np.einsum("oerdsg,odgy->yrse", Y, B, **EIN)


def row_step_right(R, T, Ak, Ab, B):
    """R[o,l,m,a] = sum R'[o',r,s,e] T[a,u,v,e] Ak[p,l,u,r,d] Ab[p,m,v,s,g] B[o,d,g,o']."""
    Y = np.einsum("yrse,auve->yrsauv", R, T, **EIN)
    Y = np.einsum("yrsauv,plurd->ysavpld", Y, Ak, **EIN)
    Y = np.einsum("ysavpld,pmvsg->yaldmg", Y, Ab, **EIN)
    return np.einsum("yaldmg,odgy->olma", Y, B, **EIN)


def two_row_step(L, T, Ak1, Ab1, Ak2, Ab2, B):
    """Column transfer through two rows:
    L'[o',r2,s2,r1,s1,e] = sum L[o,l2,m2,l1,m1,a] T[a,u1,v1,e]
        Ak1[p,l1,u1,r1,d1] Ab1[p,m1,v1,s1,g1] Ak2[q,l2,d1,r2,d2] Ab2[q,m2,g1,s2,g2] B[o,d2,g2,o']
    """
    Y = np.einsum("oLMlma,auve->oLMlmuve", L, T, **EIN)
    Y = np.einsum("oLMlmuve,plurd->oLMmveprd", Y, Ak1, **EIN)
    Y = np.einsum("oLMmveprd,pmvsg->oLMerdsg", Y, Ab1, **EIN)
    Y = np.einsum("oLMerdsg,qLdRD->oMersgqRD", Y, Ak2, **EIN)
    Y = np.einsum("oMersgqRD,qMgSG->oersRDSG", Y, Ab2, **EIN)
    return np.einsum("oersRDSG,oDGy->yRSrse", Y, B, **EIN)


def two_row_step_right(R, T, Ak1, Ab1, Ak2, Ab2, B):
    """Mirror of ``two_row_step``: R[o,l2,m2,l1,m1,a] from R'[o',r2,s2,r1,s1,e]."""
    Y = np.einsum("yRSrse,auve->yRSrsauv", R, T, **EIN)
    Y = np.einsum("yRSrsauv,plurd->yRSsavpld", Y, Ak1, **EIN)
    Y = np.einsum("yRSsavpld,pmvsg->yRSaldmg", Y, Ab1, **EIN)
    Y = np.einsum("yRSaldmg,qLdRD->ySalmgqLD", Y, Ak2, **EIN)
    Y = np.einsum("ySalmgqLD,qMgSG->yalmLDMG", Y, Ab2, **EIN)
    return np.einsum("yalmLDMG,oDGy->oLMlma", Y, B, **EIN)


def _normalised(X):
    n = float(np.sqrt(np.sum(X * X)))
    return X / n, np.log(n)


def row_environments(T, Arow, B, lam, rho):
    """Normalised left/right environments of one row and their log-scales.

    Lenv[c] closes columns < c, Renv[c] closes columns >= c (c = 0..Lc).
    """
    Lc = len(Arow)
    Dl, Dr = Arow[0].shape[1], Arow[-1].shape[3]
    Lenv = [None] * (Lc + 1)
    Renv = [None] * (Lc + 1)
    sL = np.zeros(Lc + 1)
    sR = np.zeros(Lc + 1)
    Lenv[0] = lam.reshape(1, Dl, Dl, 1)
    Renv[Lc] = rho.reshape(1, Dr, Dr, 1)
    for c in range(Lc):
        Lenv[c + 1], s = _normalised(row_step(Lenv[c], T[c], Arow[c], Arow[c], B[c]))
        sL[c + 1] = sL[c] + s
    for c in range(Lc - 1, -1, -1):
        Renv[c], s = _normalised(row_step_right(Renv[c + 1], T[c], Arow[c], Arow[c], B[c]))
        sR[c] = sR[c + 1] + s
    return Lenv, Renv, sL, sR


def row_observables(T, Arow, B, lam, rho):
    """<Sz> at every site and the horizontal bond energies of one row."""
    Lc = len(Arow)
    Lenv, Renv, sL, sR = row_environments(T, Arow, B, lam, rho)
    sz = np.zeros(Lc)
    hb = np.zeros(max(Lc - 1, 0))
    for c in range(Lc):
        A = Arow[c]
        num = np.sum(row_step(Lenv[c], T[c], apply_op(SZ, A), A, B[c]) * Renv[c + 1])
        den = np.sum(row_step(Lenv[c], T[c], A, A, B[c]) * Renv[c + 1])
        sz[c] = num / den
    for c in range(Lc - 1):
        A1, A2 = Arow[c], Arow[c + 1]
        den = np.sum(row_step(row_step(Lenv[c], T[c], A1, A1, B[c]), T[c + 1], A2, A2, B[c + 1])
                     * Renv[c + 2])
        num = 0.0
        for w, O1, O2 in BOND_TERMS:
            X = row_step(Lenv[c], T[c], apply_op(O1, A1), A1, B[c])
            X = row_step(X, T[c + 1], apply_op(O2, A2), A2, B[c + 1])
            num += w * np.sum(X * Renv[c + 2])
        hb[c] = num / den
    c = Lc // 2
    Z = float(np.sum(Lenv[c] * Renv[c]))
    return sz, hb, Z, sL[c] + sR[c], (Lenv, Renv, sL, sR)


def site_environment(T, Arow, B, lam, rho, c):
    """Norm environment of site c of one row: the network of <psi|psi> with
    the ket and bra tensors of that site taken out, the matrix N_l of the
    ALS tensor update N_l A_l = b_l (Sec. 2).

    N[l,u,r,d,m,v,s,g] = sum L[o,l,m,a] T[a,u,v,e] R[o',r,s,e] B[o,d,g,o']
    with the normalised environments L = Lenv[c], R = Renv[c+1] of the row,
    returned as a (Dl Du Dr Dd) x (Dl Du Dr Dd) matrix (ket legs as rows)
    divided by |w|, w = sum_p A[p,k] N[k,k'] A[p,k'] of this row's own
    site, with log|w| + sL[c] + sR[c+1] and the sign of w.
    """
    Lenv, Renv, sL, sR = row_environments(T, Arow, B, lam, rho)
    Y = np.einsum("olma,auve->olmuve", Lenv[c], T[c], **EIN)
    Y = np.einsum("olmuve,odgy->lmuvedgy", Y, B[c], **EIN)
    N = np.einsum("lmuvedgy,yrse->lurdmvsg", Y, Renv[c + 1], **EIN)
    _, Dl, Du, Dr, Dd = Arow[c].shape
    K = Dl * Du * Dr * Dd
    N = N.reshape(K, K)
    A = Arow[c].reshape(-1, K)
    w = float(np.einsum("pk,kj,pj->", A, N, A))
    return N / abs(w), np.log(abs(w)) + sL[c] + sR[c + 1], (1.0 if w >= 0 else -1.0)


def bond_fit_environments(T, Arow, B, lam, rho, c, G, S1, S2):
    """The two local problems of fitting G psi on the bond (c, c+1) with the
    new state psi' = psi except S1, S2 at sites c, c+1 (the alternating
    least-squares solve of the bond update, Sec. 2 and Sec. 5.2):

    N1 (S2): norm environment of site c in <psi'|psi'>,  b1 (S2) = d<psi'|G psi>/d S1,
    N2 (S1): norm environment of site c+1,                b2 (S1) = d<psi'|G psi>/d S2,

    every quantity from the normalised Lenv[c], Renv[c+2] of the row and
    divided by one number per site (the scaling of ``bond_gate_environment``),
    so that S1 = b1 N1^-1 and S2 = b2 N2^-1 solve the two problems; with
    S = A they reduce to ``site_environment`` and ``bond_gate_environment``.
    """
    Lenv, Renv, sL, sR = row_environments(T, Arow, B, lam, rho)
    bl, br = bond_gate_environment(T, Arow, B, lam, rho, c, G)   # for the scale factors below
    A1, A2 = Arow[c], Arow[c + 1]
    Theta = np.einsum("pPqQ,qQludURD->pPludURD", G, np.einsum("qlurd,QrURD->qQludURD", A1, A2, **EIN), **EIN)
    X = np.einsum("olmuve,odgy->lumvdgye", np.einsum("olma,auve->olmuve", Lenv[c], T[c], **EIN), B[c], **EIN)
    Z = np.einsum("zRSeUV,yDGz->RSeUVyDG", np.einsum("zRSf,eUVf->zRSeUV", Renv[c + 2], T[c + 1], **EIN),
                  B[c + 1], **EIN)
    E = np.einsum("lumvdgye,SeVyGpPlud->pPmvgVSG", X,
                  np.einsum("RSeUVyDG,pPludURD->SeVyGpPlud", Z, Theta, **EIN), **EIN)
    # raw environments with the substitutes in place of the other site
    R1 = row_step_right(Renv[c + 2], T[c + 1], S2, S2, B[c + 1])
    L2 = row_step(Lenv[c], T[c], S1, S1, B[c])

    def norm_env(L, k, R):
        Y = np.einsum("olma,auve->olmuve", L, T[k], **EIN)
        Y = np.einsum("olmuve,odgy->lmuvedgy", Y, B[k], **EIN)
        K = int(np.prod(Arow[k].shape[1:]))
        return np.einsum("lmuvedgy,yrse->lurdmvsg", Y, R, **EIN).reshape(K, K)

    def absw(k):
        N = norm_env(Lenv[k], k, Renv[k + 1])
        a = Arow[k].reshape(Arow[k].shape[0], -1)
        return abs(float(np.einsum("pk,kj,pj->", a, N, a)))

    sc1 = np.exp(sR[c + 1] - sR[c + 2]) * absw(c)
    sc2 = np.exp(sL[c + 1] - sL[c]) * absw(c + 1)
    N1 = norm_env(Lenv[c], c, R1) / sc1
    N2 = norm_env(L2, c + 1, Renv[c + 2]) / sc2
    b1 = np.einsum("pPmvgVSG,PsVSG->pmvsg", E, S2, **EIN).reshape(A1.shape[0], -1) / sc1
    b2 = np.einsum("pPmvgVSG,pmvsg->PsVSG", E, S1, **EIN).reshape(A2.shape[0], -1) / sc2
    return N1, b1, N2, b2


def bond_gate_environment(T, Arow, B, lam, rho, c, G):
    """Right-hand sides b of the ALS update of the horizontal bond (c, c+1)
    under a two-site gate (Sec. 2, N_l A_l = b_l): the overlap <psi'|G psi>
    with psi' = psi, differentiated by the bra tensor of site c (b_left) or
    of site c+1 (b_right).

    G[p, P, q, Q] maps the physical indices (q, Q) of sites (c, c+1) to
    (p, P).  The pair environment with both bra tensors removed is
    E[p,P,m,v,g,V,S,G'] = sum L[o,l,m,a] T_c[a,u,v,e] T_c+1[e,U,V,f]
        Theta[p,P,l,u,d,U,R,D] B_c[o,d,g,y] B_c+1[y,D,G',z] R[z,R,S,f],
    Theta = G . (A_c A_c+1) summed over the shared bond, with the normalised
    Lenv[c], Renv[c+2]; b_left = E . A_c+1 (bra), b_right = E . A_c (bra),
    each as a (d, Dl Du Dr Dd) matrix divided by the same numbers as the
    site's norm environment (``site_environment``), so that G = 1 gives
    b[p, k'] = sum_k A[p, k] N[k, k'] (k the ket, k' the bra legs).
    """
    Lenv, Renv, sL, sR = row_environments(T, Arow, B, lam, rho)
    A1, A2 = Arow[c], Arow[c + 1]
    Theta = np.einsum("pPqQ,qQludURD->pPludURD", G, np.einsum("qlurd,QrURD->qQludURD", A1, A2, **EIN), **EIN)
    X = np.einsum("olmuve,odgy->lumvdgye", np.einsum("olma,auve->olmuve", Lenv[c], T[c], **EIN), B[c], **EIN)
    Z = np.einsum("zRSeUV,yDGz->RSeUVyDG", np.einsum("zRSf,eUVf->zRSeUV", Renv[c + 2], T[c + 1], **EIN),
                  B[c + 1], **EIN)
    W = np.einsum("RSeUVyDG,pPludURD->SeVyGpPlud", Z, Theta, **EIN)
    E = np.einsum("lumvdgye,SeVyGpPlud->pPmvgVSG", X, W, **EIN)
    bl = np.einsum("pPmvgVSG,PsVSG->pmvsg", E, A2, **EIN)
    br = np.einsum("pPmvgVSG,pmvsg->PsVSG", E, A1, **EIN)

    def absw(k):   # |sum_p A N A| of site k, N from the normalised environments
        Y = np.einsum("olma,auve->olmuve", Lenv[k], T[k], **EIN)
        Y = np.einsum("olmuve,odgy->lmuvedgy", Y, B[k], **EIN)
        N = np.einsum("lmuvedgy,yrse->lurdmvsg", Y, Renv[k + 1], **EIN)
        K = int(np.prod(Arow[k].shape[1:]))
        a = Arow[k].reshape(-1, K)
        return abs(float(np.einsum("pk,kj,pj->", a, N.reshape(K, K), a)))

    sc_l = np.exp(sR[c + 1] - sR[c + 2]) * absw(c)       # Renv[c+1] = step(Renv[c+2]) / its norm
    sc_r = np.exp(sL[c + 1] - sL[c]) * absw(c + 1)       # Lenv[c+1] = step(Lenv[c]) / its norm
    return (bl.reshape(A1.shape[0], -1) / sc_l, br.reshape(A2.shape[0], -1) / sc_r)


def two_row_observables(T, Arow1, Arow2, B, lam1, rho1, lam2, rho2):
    """Vertical bond energies between two adjacent rows, per column."""
    Lc = len(Arow1)
    Dl1, Dl2 = Arow1[0].shape[1], Arow2[0].shape[1]
    Dr1, Dr2 = Arow1[-1].shape[3], Arow2[-1].shape[3]
    Lenv = [None] * (Lc + 1)
    Renv = [None] * (Lc + 1)
    Lenv[0] = np.einsum("LM,lm->LMlm", lam2, lam1).reshape(1, Dl2, Dl2, Dl1, Dl1, 1)
    Renv[Lc] = np.einsum("RS,rs->RSrs", rho2, rho1).reshape(1, Dr2, Dr2, Dr1, Dr1, 1)
    for c in range(Lc):
        A1, A2 = Arow1[c], Arow2[c]
        Lenv[c + 1], _ = _normalised(two_row_step(Lenv[c], T[c], A1, A1, A2, A2, B[c]))
    for c in range(Lc - 1, -1, -1):
        A1, A2 = Arow1[c], Arow2[c]
        Renv[c], _ = _normalised(two_row_step_right(Renv[c + 1], T[c], A1, A1, A2, A2, B[c]))
    vb = np.zeros(Lc)
    for c in range(Lc):
        A1, A2 = Arow1[c], Arow2[c]
        den = np.sum(two_row_step(Lenv[c], T[c], A1, A1, A2, A2, B[c]) * Renv[c + 1])
        num = 0.0
        for w, O1, O2 in BOND_TERMS:
            X = two_row_step(Lenv[c], T[c], apply_op(O1, A1), A1, apply_op(O2, A2), A2, B[c])
            num += w * np.sum(X * Renv[c + 1])
        vb[c] = num / den
    return vb
