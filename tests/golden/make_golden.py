"""Writes the closed-form fixtures in this folder.

Each fixture is a matrix A = Q0 R0 built from exactly representable factors:
Q0 has orthonormal columns with entries that are exact binary fractions and
R0 is an integer upper triangular matrix with a positive diagonal.  By Lemma
l_r1r2 (Section 2.1) the thin QR with positive diag(R) is unique, and by Remark
r_precond (Section 3.1) rpCholesky-QR returns that factorization whatever
nonsingular R_s the sample gives; so the expected Q and R are Q0 and R0 exactly,
independent of the seed.  No value here comes from any implementation of the
method.  Run:  python tests/golden/make_golden.py
"""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def walsh(m, cols):
    i = np.arange(m)[:, None]
    j = np.asarray(cols)[None, :]
    bits = np.vectorize(lambda x: bin(int(x)).count("1"))(i & j)
    return np.where(bits % 2 == 0, 1.0, -1.0)


def write(name, A, Q, R, s, seed, note):
    m, n = A.shape
    with open(os.path.join(HERE, name), "w") as f:
        f.write(f"# {note}\n")
        f.write("# Expected Q, R by uniqueness of the thin QR with positive diag(R) (Lemma l_r1r2,\n")
        f.write("# Section 2.1) and Remark r_precond (Section 3.1): any nonsingular R_s gives the same Q.\n")
        f.write(f"m {m}\nn {n}\ns {s}\nseed {seed}\n")
        for tag, M in (("A", A), ("Q", Q), ("R", R)):
            f.write(f"{tag}\n")
            for row in M:
                f.write(" ".join(repr(float(x)) for x in row) + "\n")


def main():
    # 16 x 4: columns 1, 2, 4, 8 of the Sylvester-Hadamard matrix H_16 scaled by 1/4
    # (entries +-0.25, every row a different sign pattern), times an integer R0.
    Q0 = walsh(16, [1, 2, 4, 8]) / 4.0
    R0 = np.array([[4, 1, -2, 3], [0, 2, 5, -1], [0, 0, 1, 2], [0, 0, 0, 8]], dtype=np.float64)
    write("walsh_16x4.txt", Q0 @ R0, Q0, R0, 12, 7,
          "A = W R0, W = columns 1,2,4,8 of the 16x16 Sylvester-Hadamard matrix / 4")
    # 4 x 1: a = (3, 4, 12, 84), ||a||_2 = 85 (3^2+4^2+12^2+84^2 = 85^2):  Q = a/85, R = 85.
    a = np.array([[3.0], [4.0], [12.0], [84.0]])
    write("pythagorean_4x1.txt", a, a / 85.0, np.array([[85.0]]), 3, 11,
          "n = 1: Q = a/||a||_2 and R = ||a||_2 with a = (3,4,12,84), ||a||_2 = 85")
    # 64 x 8: columns 1,2,4,...,128 -> 64 rows of the 64x64 Sylvester-Hadamard matrix use
    # bits 0..5 only; take columns 1,2,4,8,16,32,3,5 (Walsh functions, orthogonal) / 8.
    Q1 = walsh(64, [1, 2, 4, 8, 16, 32, 3, 5]) / 8.0
    R1 = np.triu(np.arange(1, 65, dtype=np.float64).reshape(8, 8) % 7 - 3.0)
    np.fill_diagonal(R1, [16.0, 1.0, 4.0, 2.0, 8.0, 1.0, 32.0, 1.0])
    write("walsh_64x8.txt", Q1 @ R1, Q1, R1, 24, 3,
          "A = W R1, W = Walsh columns 1,2,4,8,16,32,3,5 of the 64x64 Sylvester-Hadamard matrix / 8")


if __name__ == "__main__":
    main()
