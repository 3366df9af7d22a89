/*
 * oracle.h - TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU definition of what the LLAMA hot path computes (arXiv
 * 2302.08251): per record, per leaf field, per byte or bit.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg use it; the
 * product library never does.  It shares no code, header, table or constant
 * with the GPU library.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

enum { ORC_F32 = 0, ORC_F64, ORC_I8, ORC_U8, ORC_I16, ORC_U16, ORC_I32, ORC_U32,
       ORC_I64, ORC_U64, ORC_F16, ORC_BF16 };

enum { ORC_AOS = 0, ORC_SOA_SB, ORC_SOA_MB, ORC_AOSOA, ORC_BYTESPLIT, ORC_CHANGETYPE,
       ORC_BITPACK_INT, ORC_BITPACK_FLOAT, ORC_NULL, ORC_SPLIT, ORC_FIELD_ACCESS_COUNT,
       ORC_HEATMAP };

typedef struct orc_rec {
  uint32_t nf;
  const int* types;
} orc_rec;

typedef struct orc_map {
  int kind;
  uint32_t lanes;      /* AoSoA L; Split: fields in the first part; Heatmap: bytes per counter */
  uint32_t bits;       /* BitPackedInt B           */
  uint32_t exp_bits;   /* BitPackedFloat E         */
  uint32_t man_bits;   /* BitPackedFloat M         */
  int aos_packed;      /* AoS without padding      */
  const int* stored_types;       /* ChangeType    */
  const struct orc_map* inner;   /* Bytesplit / ChangeType / the instrumented mapping;
                                    Split: its two parts (an array of 2) */
  int round_rne;       /* BitPackedFloat: round the mantissa to nearest even
                          instead of truncating it */
} orc_map;

#endif
