"""CPU oracle of the isogeometric generation path -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may
import anything from this package.
"""
