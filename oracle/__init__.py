"""CPU oracle for the ASH hash map (test infrastructure only).

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package.  It wraps liboracle.so (ash_oracle.cpp, a sequential std::map
implementation) with numpy arrays; it shares no code with the HIP path.
"""
from .oracle import OracleMap, oracle_block_coords, oracle_voxelize, build_oracle, ORACLE_OK, ORACLE_E_INVALID, ORACLE_E_CAPACITY

__all__ = ["OracleMap", "oracle_block_coords", "oracle_voxelize", "build_oracle", "ORACLE_OK", "ORACLE_E_INVALID", "ORACLE_E_CAPACITY"]
