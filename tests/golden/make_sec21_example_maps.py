"""Writes sec21_example_maps_z3.txt: the index maps printed in the worked example of
Sec. 2.1 (w_abij = sum_kl u_abkl v_klij), evaluated at G = 3 with 0-based sectors.

The maps are the paper's own formulas, evaluated by plain integer arithmetic mod G
(no code of the oracle or of the library): the standard reduced form's implicit
sector B = I + J - A, the Alg. 1 loop bounds J = A + B - I and L = A + B - K, and
the aligned forms' B = Q - A, I = Q - J, K = Q - L.

Usage: python tests/golden/make_sec21_example_maps.py   (rewrites the file beside it)
"""
import itertools
import os

G = 3
HEADER = """\
# Index maps of the worked example of Sec. 2.1, w_abij = sum_kl u_abkl v_klij, evaluated at G = 3.
# Paper, Sec. 2.1: standard reduced forms (implicit B for w and u, implicit L for v):
#   wbar_{aA,b,iI,jJ} = w_{aA,b,I+J-A,iI,jJ};  ubar_{aA,b,kK,lL} = u_{aA,b,K+L-A,kK,lL};
#   vbar_{kK,l,iI,jJ} = v_{kK,l,I+J-K,iI,jJ}
# Alg. 1 loop nest: J = A+B-I, L = A+B-K.
# Aligned forms with auxiliary Q = I+J = A+B = K+L (mod G):
#   what_{aA,b,i,jJ,Q} = w_{aA,b,Q-A,i,Q-J,jJ};  uhat_{aA,b,k,lL,Q} = u_{aA,b,Q-A,k,Q-L,lL};
#   vhat_{k,lL,i,jJ,Q} = v_{k,Q-L,lL,i,Q-J,jJ}
# Every sign string is ++-- with total charge 0.  Sectors are 0-based here.
# Rows 'std X Y Z -> B' : (A, I, J) -> implicit B of wbar; (A, K, L) -> implicit B of ubar.
# Rows 'alg1 A B I K -> J L'.
# Rows 'aligned Q A J L -> B I K' : B = Q-A, I = Q-J, K = Q-L.
"""


def lines():
    out = []
    for A, I, J in itertools.product(range(G), repeat=3):
        out.append(f"std {A} {I} {J} -> {(I + J - A) % G}")
    for A, B, I, K in itertools.product(range(G), repeat=4):
        out.append(f"alg1 {A} {B} {I} {K} -> {(A + B - I) % G} {(A + B - K) % G}")
    for Q, A, J, L in itertools.product(range(G), repeat=4):
        out.append(f"aligned {Q} {A} {J} {L} -> {(Q - A) % G} {(Q - J) % G} {(Q - L) % G}")
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sec21_example_maps_z3.txt")
    with open(path, "w") as f:
        f.write(HEADER + "\n".join(lines()) + "\n")
