// Input front end (host only): FASTA / FASTQ text -> the read layout the
// insert calls take (sequence bytes concatenated, CSR offsets).
#include <cstring>

#include "kmerco.h"

namespace {

// One line of text[pos, len): [b, e) without the line end ("\n", "\r\n");
// pos moves past the line end.
struct Lines {
    const char *text;
    uint64_t len, pos = 0;

    bool next(uint64_t &b, uint64_t &e) {
        if (pos >= len)
            return false;
        b = pos;
        const void *nl = std::memchr(text + pos, '\n', (size_t)(len - pos));
        uint64_t end = nl ? (uint64_t)((const char *)nl - text) : len;
        pos = nl ? end + 1 : len;
        e = end;
        if (e > b && text[e - 1] == '\r')
            e--;
        return true;
    }
};

// Output with capacities: counts always advance, bytes are written only
// inside the capacity.
struct Out {
    uint8_t *seq;
    uint64_t seq_cap;
    uint64_t *off;
    uint64_t off_cap;
    uint64_t n_bases = 0, n_reads = 0;

    void bases(const char *p, uint64_t n) {
        if (n && n_bases < seq_cap) {
            const uint64_t room = seq_cap - n_bases;
            std::memcpy(seq + n_bases, p, (size_t)(n < room ? n : room));
        }
        n_bases += n;
    }
    void end_read() {
        n_reads++;
        if (n_reads < off_cap)
            off[n_reads] = n_bases;
    }
};

}  // namespace

extern "C" {

kc_status kc_parse_fastx(const char *text, uint64_t len, uint32_t flags, uint8_t *seq,
                         uint64_t seq_cap, uint64_t *offsets, uint64_t off_cap,
                         uint64_t *n_bases, uint64_t *n_reads) {
    if ((len && !text) || (seq_cap && !seq) || (off_cap && !offsets) || !n_bases || !n_reads ||
        (flags & ~(uint32_t)KC_FASTX_ONE_SEQUENCE))
        return KC_EINVAL;
    const bool one = (flags & KC_FASTX_ONE_SEQUENCE) != 0;
    Out o{seq, seq_cap, offsets, off_cap};
    if (off_cap)
        offsets[0] = 0;
    Lines L{text, len};
    uint64_t b, e;
    // the format is the first line's that is neither blank nor a comment
    char fmt = 0;
    uint64_t first = 0;
    while (L.next(b, e)) {
        if (e > b && text[b] != ';') {
            fmt = text[b];
            first = b;
            break;
        }
    }
    kc_status st = KC_OK;
    uint64_t records = 0;
    if (fmt == '>') {
        L.pos = first;
        bool open = false;
        while (L.next(b, e)) {
            if (e == b || text[b] == ';')
                continue;  // blank line, comment
            if (text[b] == '>') {
                if (open && !one)
                    o.end_read();
                open = true;
                records++;
                continue;
            }
            o.bases(text + b, e - b);
        }
        if (open && !one)
            o.end_read();
    } else if (fmt == '@') {
        L.pos = first;
        while (st == KC_OK && L.next(b, e)) {
            if (e == b)
                continue;  // blank line between records
            if (text[b] != '@') {
                st = KC_EINVAL;
                break;
            }
            records++;
            // sequence lines up to the '+' line
            uint64_t n_seq = 0;
            bool plus = false;
            while (L.next(b, e)) {
                if (e > b && text[b] == '+') {
                    plus = true;
                    break;
                }
                o.bases(text + b, e - b);
                n_seq += e - b;
            }
            if (!plus) {
                st = KC_EINVAL;
                break;
            }
            // quality lines of the same total length (they may start with '@')
            uint64_t n_q = 0;
            while (n_q < n_seq && L.next(b, e))
                n_q += e - b;
            if (n_q != n_seq) {
                st = KC_EINVAL;
                break;
            }
            if (!one)
                o.end_read();
        }
    } else if (fmt != 0) {
        st = KC_EINVAL;
    }
    if (st != KC_OK)
        return st;
    if (one && records)
        o.end_read();
    *n_bases = o.n_bases;
    *n_reads = o.n_reads;
    return (o.n_bases > seq_cap || o.n_reads + 1 > off_cap) ? KC_ERANGE : KC_OK;
}

}  // extern "C"
