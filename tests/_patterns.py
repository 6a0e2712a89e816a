"""Circuit patterns shared by the host and GPU tests (gate lists only)."""
from workloads import circuits as C


def cnot_pattern(n, kind):
    """Circuits whose CNOT structure exercises the folding of CNOTs into LDS
    remaps: runs at the start and the end, ZZ-type CNOT-RZ-CNOT sandwiches,
    pairs that cancel, and rings."""
    b = C._Builder(n)

    def rots():
        for q in range(n):
            b.rot("RY", q, p_w=b.new_param())
            b.rot("RZ", q, p_w=b.new_param())

    def chain():
        for q in range(n - 1):
            b.fixed("CNOT", q, q + 1)

    def ring():
        for q in range(n):
            b.fixed("CNOT", q, (q + 1) % n)

    if kind == "start_end":
        chain(); rots(); ring(); rots(); chain()
    elif kind == "zz":
        rots()
        for q in range(n - 1):
            b.fixed("CNOT", q, q + 1)
            b.rot("RZ", q + 1, p_w=b.new_param())
            b.fixed("CNOT", q, q + 1)
        rots()
    elif kind == "cancel":
        rots()
        for q in range(n - 1):
            b.fixed("CNOT", q, q + 1)
            b.fixed("CNOT", q, q + 1)
        rots()
        ring()
        b.fixed("CZ", 0, n - 1)
        rots()
    else:  # only CNOTs
        chain(); ring(); chain()
    return b.build()
